// Device helpers shared by the kernel translation units: global-memory views,
// the encode/lift helpers of the packed encodings, the multiply-accumulate
// operand form, block-to-work maps and the NTT launch dispatch.
#pragma once
#include "pencil_internal.h"
#include "modarith.h"

namespace pencil {

// Global-memory views of generic pointers.  Pointers read from device memory
// (the batched step's segment tables) are generic to the compiler, which then
// emits flat instructions; flat loads also count against the LDS/scalar wait
// counter.  Every buffer here is global memory, so the hot loops access it
// through these address-space-qualified views.
#define PENCIL_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ PENCIL_GLOBAL T* gview(T* p) {
  return (PENCIL_GLOBAL T*)p;
}
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// Split form of a residue v < 2^60, the multiply-accumulate's operand format
// (and the format of the data owner's NTT-domain ciphertexts):
// (v mod 2^30) | (v >> 30) << 32.
__device__ __forceinline__ uint64_t split30(uint64_t v) { return (v & 0x3FFFFFFFull) | ((v >> 30) << 32); }
__device__ __forceinline__ uint64_t unsplit30(uint64_t s) { return (s & 0xFFFFFFFFull) | ((s >> 32) << 30); }

// ---------------------------------------------------------- encode helpers
// round(q m / t) mod q_l for m in [0, t): Delta * m + round(rho m / t), rho = q mod t.
__device__ __forceinline__ uint64_t round_rho(uint64_t m, const Consts& C) {
  uint64_t est = __umul64hi(m, C.rho_sh);
  uint64_t r = m * C.rho - est * C.t;  // in [0, 2t)
  if (r >= C.t) {
    r -= C.t;
    est += 1;
  }
  return est + (2 * r > C.t ? 1 : 0);
}

__device__ __forceinline__ uint64_t delta_scale(uint64_t m, uint64_t rr, const LimbConst& lc) {
  return add_mod(mul_shoup(m, lc.delta, lc.delta_sh, lc.q), rr, lc.q);
}

// floor(n / d) for n, d < 2^16 from m = ceil(2^32 / d) (m = 0 stands for
// d = 1): rounding the reciprocal up adds less than n / 2^32 < 2^-16 to n / d,
// whose fractional part is at most 1 - 1/d <= 1 - 2^-16, so the floor holds.
__device__ __forceinline__ int fdiv(int n, uint32_t m) { return m ? (int)__umulhi((uint32_t)n, m) : n; }

// Origin of one operand tile in virtual coordinates, decoded once per tile:
// A side (m, k, y, x) of slot 0's entry; K side (r, k, kernel row, kernel column).
struct TileOrigin {
  int i0, i1, y, x;
};

// A tiles are numbered ((((mi*nK + ki)*nOY + oyi)*nOX + oxi)*nKY + kyi)*nKX + kxi.
__device__ __forceinline__ TileOrigin a_tile_origin(const Geo& G, int64_t tile) {
  int64_t ti = tile;
  const int kxi = (int)(ti % G.nKX); ti /= G.nKX;
  const int kyi = (int)(ti % G.nKY); ti /= G.nKY;
  const int oxi = (int)(ti % G.nOX); ti /= G.nOX;
  const int oyi = (int)(ti % G.nOY); ti /= G.nOY;
  const int ki = (int)(ti % G.nK); ti /= G.nK;
  const int mi = (int)ti;
  return {mi * G.mt, ki * G.kt, oyi * G.oh + kyi * G.kh, oxi * G.ow + kxi * G.kw};
}

// K tiles are numbered ((ri*nK + ki)*nKY + kyi)*nKX + kxi.
__device__ __forceinline__ TileOrigin k_tile_origin(const Geo& G, int64_t tile) {
  int64_t ti = tile;
  const int kxi = (int)(ti % G.nKX); ti /= G.nKX;
  const int kyi = (int)(ti % G.nKY); ti /= G.nKY;
  const int ki = (int)(ti % G.nK); ti /= G.nK;
  const int ri = (int)ti;
  return {ri * G.rt, ki * G.kt, kyi * G.kh, kxi * G.kw};
}

__device__ __forceinline__ TileOrigin tile_origin(int side, const Geo& G, int64_t tile) {
  return side == 0 ? a_tile_origin(G, tile) : k_tile_origin(G, tile);
}

// Offset into the caller's tensor of the forward-encoded A tile's value at
// polynomial slot `slot` (App. A's pi_v generalised: slot = mm*RS + kk*ha*wa +
// ya*wa + xa), or -1 for an empty slot.
__device__ __forceinline__ int64_t a_slot_at(const Geo& G, const View& V, const TileOrigin& T, int slot) {
  const int mm = fdiv(slot, G.dv_rs);
  const int rem = slot - mm * G.RS;
  if (mm >= G.mt || rem >= G.S) return -1;
  const int hw = G.ha * G.wa;
  const int kk = fdiv(rem, G.dv_hw);
  const int rem2 = rem - kk * hw;
  const int ya = fdiv(rem2, G.dv_wa), xa = rem2 - ya * G.wa;
  const int m = T.i0 + mm, k = T.i1 + kk, y = T.y + ya, x = T.x + xa;
  if (m >= G.M || k >= G.K || y >= G.HA || x >= G.WA) return -1;
  const int ys = y - V.pady, xs = x - V.pad;
  if (ys < 0 || xs < 0 || ys >= V.H || xs >= V.W) return -1;
  return m * V.s0 + k * V.s1 + ys * V.sy + xs * V.sx;
}

// The same for the reverse-encoded K tile (App. A's pi_W: slot = O + rr*S -
// (kk*ha*wa + dy*wa + dx)).
__device__ __forceinline__ int64_t k_slot_at(const Geo& G, const View& V, const TileOrigin& T, int slot) {
  const int z = slot - G.O + G.S - 1;
  if (z < 0) return -1;
  const int rr = fdiv(z, G.dv_s);
  if (rr >= G.rt) return -1;
  const int D = rr * G.S + G.O - slot;  // in [0, S)
  const int hw = G.ha * G.wa;
  const int kk = fdiv(D, G.dv_hw);
  const int rem = D - kk * hw;
  const int dy = fdiv(rem, G.dv_wa), dx = rem - dy * G.wa;
  if (dy >= G.kh || dx >= G.kw) return -1;
  const int r = T.i0 + rr, k = T.i1 + kk;
  int a = T.y + dy, b = T.x + dx;
  if (r >= G.R || k >= G.K || a >= G.KH || b >= G.KW) return -1;
  if (V.flip) {
    a = V.KH - 1 - a;
    b = V.KW - 1 - b;
  }
  return r * V.s0 + k * V.s1 + a * V.sy + b * V.sx;
}

// Entry e of a reverse-encoded K tile, e = ((rr kt + kk) kh + dy) kw + dx over
// rr < rt, kk < kt, dy < kh, dx < kw (every K-tile slot that k_slot_at maps
// to the tensor is one such entry, and each entry has one slot): its slot
// O + rr S - (kk ha wa + dy wa + dx) and the tensor offset of its value, or
// -1 for an entry past the tensor (a ragged tile).
__device__ __forceinline__ int64_t k_entry_at(const Geo& G, const View& V, const TileOrigin& T, int e, int& slot) {
  const int thw = G.kt * G.kh * G.kw, hw = G.kh * G.kw;
  const int rr = fdiv(e, G.dv_kthw);
  const int rem = e - rr * thw;
  const int kk = fdiv(rem, G.dv_khw);
  const int rem2 = rem - kk * hw;
  const int dy = fdiv(rem2, G.dv_kw), dx = rem2 - dy * G.kw;
  slot = G.O + rr * G.S - (kk * G.ha * G.wa + dy * G.wa + dx);
  const int r = T.i0 + rr, k = T.i1 + kk;
  int a = T.y + dy, b = T.x + dx;
  if (r >= G.R || k >= G.K || a >= G.KH || b >= G.KW) return -1;
  if (V.flip) {
    a = V.KH - 1 - a;
    b = V.KW - 1 - b;
  }
  return r * V.s0 + k * V.s1 + a * V.sy + b * V.sx;
}

__device__ __forceinline__ int64_t slot_at(int side, const Geo& G, const View& V, const TileOrigin& T, int slot) {
  return side == 0 ? a_slot_at(G, V, T, slot) : k_slot_at(G, V, T, slot);
}

// Work item of block `b` of `total`.  Workgroups go to the 8 XCDs round-robin
// by block index, so XCD x = b mod 8 receives blocks b = x, x + 8, ...; giving
// it the contiguous work range [x total / 8, (x + 1) total / 8) in order keeps
// the chunks of one slot range (which share operands) on one L2.
__device__ __forceinline__ int64_t xcd_work(int64_t b, int64_t total) {
  const int64_t q = total >> 3, r = total & 7, x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// Segment of a batched step's phase launch that block b belongs to.
__device__ __forceinline__ int find_seg(const StepSeg* segs, int nseg, int64_t b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].block_begin <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

static inline size_t lds_bytes(const Consts& C) { return (size_t)(C.n + (C.n >> 5)) * sizeof(uint64_t); }

// Instantiate `kern<LOGN>` for the context's degree and launch it.
#define NTT_CASE(kern, LN, LE, grid, C, s, ...)                                                 \
  case (LN) * 8 + (LE):                                                                          \
    hipLaunchKernelGGL((kern<LN, LE>), grid, dim3((1u << (LN)) >> (LE)), lds_bytes(C), s, __VA_ARGS__); \
    break;
// Instantiate `kern<LOGN, LOGE>` for the context's degree and per-thread width.
#define NTT_DISPATCH(kern, grid, C, s, ...)                                                \
  do {                                                                                     \
    switch ((C).log2n * 8 + (C).ntt_loge) {                                                \
      NTT_CASE(kern, 10, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 11, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 12, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 12, 5, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 13, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 13, 5, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 14, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 14, 5, grid, C, s, __VA_ARGS__)                                       \
      default: return hipErrorInvalidValue;                                                \
    }                                                                                      \
  } while (0)

}  // namespace pencil
