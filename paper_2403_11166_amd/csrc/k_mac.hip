// Pointwise multiply-accumulate of the product path (per call and batched).
#include "device_common.h"

namespace pencil {

// LDS-staged multiply-accumulate.  The forward NTTs of the product path store
// each residue v < 2^61 split as (v mod 2^30) | (v >> 30) << 32, so a modular
// product-accumulate is four 32 x 32 -> 64-bit multiply-adds into three 64-bit
// partial sums (low x low, cross terms, high x high).  Every `mac_fold` steps
// the partial sums fold into a 128-bit total, which is Barrett-reduced every
// `mac_chunk` folds and at the end.
//
// A block owns 64 NTT slots of one limb and a ROWS x COLS chunk of (A-row,
// K-row) output tiles.  It walks the contraction (product terms x contraction
// tiles) KB steps at a time: all 512 threads first stage the chunk's A and K
// values of KB steps for their 64 slots in LDS, then each wave accumulates a
// 2 x 2 block of its slot's outputs (both components).  Chunk shapes are
// schedule variants with the same result: 0 = 4 x 8, 1 = 2 x 16, 2 = 8 x 4.
// Staging addresses advance by precomputed strides (no division per step).
constexpr int kMacSlots = 64, kMacKB = 4;
constexpr int kMacSmemWords = kMacKB * 2 * 18 * kMacSlots;  // ROWS + COLS <= 18

struct Acc {
  uint64_t s0, s1, s2;  // partial sums of a0 b0, a0 b1 + a1 b0, a1 b1
  uint64_t lo, hi;      // folded 128-bit total
};

__device__ __forceinline__ void acc_mac(Acc& x, uint64_t a, uint64_t b) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  x.s0 += (uint64_t)a0 * b0;
  x.s1 += (uint64_t)a0 * b1;
  // keeps the two middle products as two multiply-adds into s1 (summing them
  // first would cost a separate 64-bit add)
  asm volatile("" : "+v"(x.s1));
  x.s1 += (uint64_t)a1 * b0;
  x.s2 += (uint64_t)a1 * b1;
}

// total += s0 + s1 2^30 + s2 2^60; the partial sums restart at zero.
__device__ __forceinline__ void acc_fold(Acc& x) {
  const uint64_t t1 = x.s1 << 30, t2 = x.s2 << 60;
  uint64_t lo = x.lo + x.s0;
  uint64_t c = lo < x.s0 ? 1 : 0;
  lo += t1;
  c += lo < t1 ? 1 : 0;
  lo += t2;
  c += lo < t2 ? 1 : 0;
  x.hi += c + (x.s1 >> 34) + (x.s2 >> 4);
  x.lo = lo;
  x.s0 = x.s1 = x.s2 = 0;
}

// Fold every accumulator of a wave's block (every mac_fold steps) and
// Barrett-reduce one of them: accumulator i at fold i of each period of
// mac_chunk folds (mac_chunk >= 8 >= the accumulator count), so each total is
// reduced once per period while only one reduction's temporaries are live.
template <int TM, int TR, int NC>
__device__ __forceinline__ void acc_fold_all(Acc (&acc)[TM][TR][NC], uint32_t& nfold, uint32_t reduce_every,
                                             const LimbConst& lc) {
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c2 = 0; c2 < TR; ++c2)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc_fold(acc[a][c2][c]);
  const uint32_t f = nfold;
  nfold = f + 1 == reduce_every ? 0 : f + 1;
  switch (f) {
#define PENCIL_REDUCE_CASE(i)                                                    \
  case i:                                                                        \
    if (i < TM * TR * NC) {                                                      \
      Acc& x = acc[(i / (NC * TR)) % TM][(i / NC) % TR][i % NC];                  \
      x.lo = reduce128(x.hi, x.lo, lc.q, lc.mu_lo, lc.mu_hi);                     \
      x.hi = 0;                                                                  \
    }                                                                            \
    break;
    PENCIL_REDUCE_CASE(0)
    PENCIL_REDUCE_CASE(1)
    PENCIL_REDUCE_CASE(2)
    PENCIL_REDUCE_CASE(3)
    PENCIL_REDUCE_CASE(4)
    PENCIL_REDUCE_CASE(5)
    PENCIL_REDUCE_CASE(6)
    PENCIL_REDUCE_CASE(7)
#undef PENCIL_REDUCE_CASE
    default: break;
  }
}

// Loop-invariant facts of one block's share of the multiply-accumulate.
struct MacBlock {
  int64_t ln;           // limb * n + first slot of the block
  int64_t ct_stride, pt_stride;
  int row0, col0;       // chunk origin
  int rg, cg;           // this wave's first row and column in the chunk
  int s, grp;           // lane slot, wave index
  int comp;             // the ciphertext component of a one-component wave
  bool active;          // this wave's 2 x 2 block holds at least one real output
  uint32_t nmac, nfold; // steps since the last fold, folds since the last reduction
};

template <int ROWS, int COLS, bool A_CT>
__device__ __forceinline__ void mac_term(uint64_t* smem, const MacTerm& T, const MacArgs& A, const Geo& G,
                                         const Consts& C, const LimbConst& lc, MacBlock& B, Acc (&acc)[2][2][2]) {
  constexpr int TM = 2, TR = 2, KB = kMacKB;
  constexpr int KC = COLS > 8 ? 2 : 1;  // K columns staged per wave
  uint64_t(*sa)[2][ROWS][kMacSlots] = reinterpret_cast<uint64_t(*)[2][ROWS][kMacSlots]>(smem);
  uint64_t(*sk)[2][COLS][kMacSlots] =
      reinterpret_cast<uint64_t(*)[2][COLS][kMacSlots]>(smem + KB * 2 * ROWS * kMacSlots);
  const int sp = G.nOY * G.nOX, kspan = G.nKY * G.nKX;
  const int ksteps = G.nK * kspan;
  const int64_t sa_str = A_CT ? B.ct_stride : B.pt_stride, sk_str = A_CT ? B.pt_stride : B.ct_stride;
  const int grp = B.grp, s = B.s;
  // The A row this wave stages: tile index ((mi nK + ki) sp + rsp) kspan + kk
  // = arow + ki sp kspan + kk, with arow = (mi nK sp + rsp) kspan.
  const int srow = B.row0 + grp;
  const bool have_a = grp < ROWS && srow < A.m_rows;
  const PENCIL_GLOBAL uint64_t* pa = gview(T.a) + B.ln + s;
  if (have_a) {
    const int mi = srow / sp, rsp = srow % sp;
    pa += (((int64_t)mi * G.nK * sp + rsp) * kspan) * sa_str;
  }
  const int64_t a_step = sa_str, a_wrap = ((int64_t)(sp - 1) * kspan + 1) * sa_str;
  // The K columns this wave stages: tile index col ksteps + (ki kspan + kk).
  bool have_k[KC];
  const PENCIL_GLOBAL uint64_t* pk[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    const int cc = grp + 8 * j, col = B.col0 + cc;
    have_k[j] = cc < COLS && col < G.nR;
    pk[j] = gview(T.k) + B.ln + s + (have_k[j] ? (int64_t)col * ksteps * sk_str : 0);
  }
  const uint32_t fold_every = C.mac_fold, reduce_every = C.mac_chunk;
  int kk = 0;
  for (int k0 = 0; k0 < ksteps; k0 += KB) {
    __syncthreads();
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      if (k0 + b < ksteps) {
        if (have_a) {
          sa[b][0][grp][s] = pa[0];
          if (A_CT) sa[b][1][grp][s] = pa[T.c1];
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          if (have_k[j]) {
            sk[b][0][grp + 8 * j][s] = pk[j][0];
            if (!A_CT) sk[b][1][grp + 8 * j][s] = pk[j][T.c1];
          }
          pk[j] += sk_str;
        }
        if (++kk == kspan) {
          kk = 0;
          pa += a_wrap;
        } else {
          pa += a_step;
        }
      }
    }
    __syncthreads();
    if (!B.active) continue;
#pragma unroll 1
    for (int b = 0; b < KB; ++b) {
      if (k0 + b >= ksteps) break;
      uint64_t av[TM][2], kv[TR][2];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        av[a][0] = sa[b][0][B.rg + a][s];
        av[a][1] = A_CT ? sa[b][1][B.rg + a][s] : av[a][0];
      }
#pragma unroll
      for (int c2 = 0; c2 < TR; ++c2) {
        kv[c2][0] = sk[b][0][B.cg + c2][s];
        kv[c2][1] = A_CT ? kv[c2][0] : sk[b][1][B.cg + c2][s];
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c2 = 0; c2 < TR; ++c2)
#pragma unroll
          for (int c = 0; c < 2; ++c) acc_mac(acc[a][c2][c], av[a][c], kv[c2][c]);
      if (++B.nmac == fold_every) {
        B.nmac = 0;
        acc_fold_all<TM, TR, 2>(acc, B.nfold, reduce_every, lc);
      }
    }
  }
}

template <int TM, int TR, int NC, bool A_CT>
__device__ __forceinline__ void mac_term_direct(const MacTerm& T, const MacArgs& A, const Geo& G, const Consts& C,
                                                const LimbConst& lc, MacBlock& B, Acc (&acc)[TM][TR][NC]);

// One block's multiply-accumulate: chunk ROWS x COLS, each wave a TM x TR
// block of it for both ciphertext components (NC = 2) or one (NC = 1, the
// block's waves alternate components); operands staged in LDS or (DIRECT)
// loaded by each wave.
template <int ROWS, int COLS, int TM, int TR, int NC, bool DIRECT>
__device__ __forceinline__ void do_mac_t(uint64_t* smem, const MacArgs& A, const Geo& G, const Consts& C,
                                         int slot_block, int chunk) {
  constexpr int WC = COLS / TR;
  static_assert(DIRECT || (TM == 2 && TR == 2 && NC == 2), "LDS staging uses 2 x 2 two-component wave blocks");
  static_assert((ROWS / TM) * WC * (2 / NC) == 8, "8 waves per block");
  static_assert(ROWS + COLS <= 18 && ROWS <= 8 && COLS <= 16, "staging layout");
  const int n = C.n, L = C.L;
  const int per_limb = n / kMacSlots;
  const int l = slot_block / per_limb;
  const LimbConst& lc = C.limb[l];
  const int cchunks = (G.nR + COLS - 1) / COLS;
  MacBlock B;
  B.row0 = (chunk / cchunks) * ROWS;
  B.col0 = (chunk % cchunks) * COLS;
  B.s = threadIdx.x & (kMacSlots - 1);
  // wave-uniform: the row and column bookkeeping below runs on the scalar unit
  B.grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  B.comp = NC == 1 ? (B.grp & 1) : 0;
  const int tile = NC == 1 ? B.grp >> 1 : B.grp;
  B.rg = (tile / WC) * TM;
  B.cg = (tile % WC) * TR;
  B.ln = (int64_t)l * n + (int64_t)(slot_block % per_limb) * kMacSlots;
  B.ct_stride = 2 * (int64_t)L * n;
  B.pt_stride = (int64_t)L * n;
  B.active = B.row0 + B.rg < A.m_rows && B.col0 + B.cg < G.nR;
  B.nmac = B.nfold = 0;

  Acc acc[TM][TR][NC];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TR; ++b)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[a][b][c] = Acc{0, 0, 0, 0, 0};
  // term 0 has the ciphertext on the A side; a second term (the weight
  // gradient's) has it on the K side
  if constexpr (DIRECT) {
    if (!B.active) return;
    mac_term_direct<TM, TR, NC, true>(A.term[0], A, G, C, lc, B, acc);
    if (A.n_terms > 1) mac_term_direct<TM, TR, NC, false>(A.term[1], A, G, C, lc, B, acc);
  } else {
    mac_term<ROWS, COLS, true>(smem, A.term[0], A, G, C, lc, B, acc);
    if (A.n_terms > 1) mac_term<ROWS, COLS, false>(smem, A.term[1], A, G, C, lc, B, acc);
  }
  if (!B.active) return;
  // re-randomisation term pk_c * u'_o, reduction and store
  const int64_t ln = B.ln, pt_stride = B.pt_stride, ct_stride = B.ct_stride;
  const int s = B.s, sp = G.nOY * G.nOX;
  const PENCIL_GLOBAL uint64_t* gpk = gview(A.pk);
  const PENCIL_GLOBAL uint64_t* gu = gview(A.u);
  PENCIL_GLOBAL uint64_t* gout = gview(A.out);
  const uint64_t pk0 = gpk[ln + s], pk1 = gpk[pt_stride + ln + s];
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int row = B.row0 + B.rg + a;
    if (row >= A.m_rows) continue;
    const int mi = row / sp, oyi = (row % sp) / G.nOX, oxi = row % G.nOX;
#pragma unroll
    for (int b = 0; b < TR; ++b) {
      const int col = B.col0 + B.cg + b;
      if (col >= G.nR) continue;
      const int64_t o = (((int64_t)mi * G.nR + col) * G.nOY + oyi) * G.nOX + oxi;
      const uint64_t u = gu[o * pt_stride + ln + s];
#pragma unroll
      for (int ci = 0; ci < NC; ++ci) {
        // one more step (the partial sums hold fewer than mac_fold steps)
        const int c = NC == 1 ? B.comp : ci;
        Acc& x = acc[a][b][ci];
        acc_mac(x, c ? pk1 : pk0, u);
        acc_fold(x);
        gout[o * ct_stride + (int64_t)c * pt_stride + ln + s] = reduce128(x.hi, x.lo, lc.q, lc.mu_lo, lc.mu_hi);
      }
    }
  }
}

// The same chunks without LDS: each wave loads the operands of its 2 x 2 block
// straight from memory (the block's other waves read the same rows and columns
// through L1) with the next step's loads in flight while the current step is
// accumulated.  No barriers, so waves run independently.
template <int TM, int TR, int NC, bool A_CT>
__device__ __forceinline__ void mac_term_direct(const MacTerm& T, const MacArgs& A, const Geo& G, const Consts& C,
                                                const LimbConst& lc, MacBlock& B, Acc (&acc)[TM][TR][NC]) {
  const int sp = G.nOY * G.nOX, kspan = G.nKY * G.nKX;
  const int ksteps = G.nK * kspan;
  const int64_t sa_str = A_CT ? B.ct_stride : B.pt_stride, sk_str = A_CT ? B.pt_stride : B.ct_stride;
  const int64_t c1 = T.c1;
  // Rows or columns past the end read row 0 / column 0 of the chunk instead
  // (valid memory); their sums are never stored.
  const PENCIL_GLOBAL uint64_t* pa[TM];
  const PENCIL_GLOBAL uint64_t* pk[TR];
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    int row = B.row0 + B.rg + a;
    if (row >= A.m_rows) row = B.row0 + B.rg;
    const int mi = row / sp, rsp = row % sp;
    pa[a] = gview(T.a) + B.ln + B.s + (((int64_t)mi * G.nK * sp + rsp) * kspan) * sa_str;
    if (NC == 1 && A_CT) pa[a] += B.comp * c1;  // this wave's component
  }
#pragma unroll
  for (int c2 = 0; c2 < TR; ++c2) {
    int col = B.col0 + B.cg + c2;
    if (col >= G.nR) col = B.col0 + B.cg;
    pk[c2] = gview(T.k) + B.ln + B.s + (int64_t)col * ksteps * sk_str;
    if (NC == 1 && !A_CT) pk[c2] += B.comp * c1;
  }
  const int64_t a_wrap = ((int64_t)(sp - 1) * kspan + 1) * sa_str;
  const uint32_t fold_every = C.mac_fold, reduce_every = C.mac_chunk;
  int kk = 0, left = ksteps;  // steps not yet loaded
  // Four operand sets rotate so that the loads of the next three steps are in
  // flight while the current one accumulates (no register copies between
  // them).  Loads are unconditional: past the last step the pointers stop
  // advancing and the last step is read again, so no branch separates a load
  // from its use.
  uint64_t xa[TM][NC], xk[TR][NC], ya[TM][NC], yk[TR][NC], za[TM][NC], zk[TR][NC], wa[TM][NC], wk[TR][NC];
  auto load = [&](uint64_t(&va)[TM][NC], uint64_t(&vk)[TR][NC]) {
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      va[a][0] = pa[a][0];
      if (NC == 2) va[a][NC - 1] = A_CT ? pa[a][c1] : va[a][0];
    }
#pragma unroll
    for (int c2 = 0; c2 < TR; ++c2) {
      vk[c2][0] = pk[c2][0];
      if (NC == 2) vk[c2][NC - 1] = A_CT ? vk[c2][0] : pk[c2][c1];
    }
    const bool adv = --left > 0;
    const int64_t da = !adv ? 0 : (kk + 1 == kspan) ? a_wrap : sa_str;
    const int64_t dk = adv ? sk_str : 0;
    kk = (kk + 1 == kspan) ? 0 : kk + 1;
#pragma unroll
    for (int a = 0; a < TM; ++a) pa[a] += da;
#pragma unroll
    for (int c2 = 0; c2 < TR; ++c2) pk[c2] += dk;
  };
  auto step = [&](const uint64_t(&va)[TM][NC], const uint64_t(&vk)[TR][NC]) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int c2 = 0; c2 < TR; ++c2)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc_mac(acc[a][c2][c], va[a][c], vk[c2][c]);
    if (++B.nmac == fold_every) {
      B.nmac = 0;
      acc_fold_all<TM, TR, NC>(acc, B.nfold, reduce_every, lc);
    }
  };
  load(xa, xk);
  load(ya, yk);
  load(za, zk);
  for (int k = 0; k < ksteps; k += 4) {
    load(wa, wk);
    step(xa, xk);
    if (k + 1 >= ksteps) break;
    load(xa, xk);
    step(ya, yk);
    if (k + 2 >= ksteps) break;
    load(ya, yk);
    step(za, zk);
    if (k + 3 >= ksteps) break;
    load(za, zk);
    step(wa, wk);
  }
}

// ------------------------------------------------------------------ kind 1
// Direct loads, each wave a 2 x 2 block of (A row, K row) outputs for both
// ciphertext components, with the 128-bit totals kept in LDS: each lane owns
// its 16-byte words in a region private to its wave, so no barrier is needed,
// and a wave holds only the 64-bit partial sums of its 8 outputs in
// registers.  With SPLIT the two cross products a0 b1 and a1 b0 go to
// separate partial sums, so every partial sum gains one product below 2^60 per
// step and a fold is due every mac_fold4 steps (16 for 60-bit primes) instead
// of every mac_fold (8): fewer folds for 16 more registers, which the batched
// step's kernel can spend and the per-call kernel (whose by-value arguments
// hold more scalar registers) cannot without losing occupancy.
template <bool SPLIT>
struct Part {
  uint64_t s0, s1, s1b, s2;  // partial sums of a0 b0, a0 b1 (+ a1 b0 unless SPLIT), a1 b0, a1 b1
};
template <>
struct Part<false> {
  uint64_t s0, s1, s2;
};

template <bool SPLIT>
__device__ __forceinline__ void part_mac(Part<SPLIT>& x, uint64_t a, uint64_t b) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  x.s0 += (uint64_t)a0 * b0;
  x.s1 += (uint64_t)a0 * b1;
  if constexpr (SPLIT) {
    x.s1b += (uint64_t)a1 * b0;
  } else {
    // two multiply-adds into s1 (summing the products first would cost a 64-bit add)
    asm volatile("" : "+v"(x.s1));
    x.s1 += (uint64_t)a1 * b0;
  }
  x.s2 += (uint64_t)a1 * b1;
}

// (lo, hi) += s0 + (s1 [+ s1b]) 2^30 + s2 2^60; the partial sums restart at
// zero.  The fold is formed as a 128-bit value (flo, fhi) in 64-bit pieces:
// with a = s1 + s1b = a' + ca 2^64, a 2^30 is (a' << 30) below 2^64 and
// (a' >> 34) + ca 2^30 above; s2 2^60 is (s2 << 60) below and s2 >> 4 above.
// The total never wraps.
template <bool SPLIT>
__device__ __forceinline__ void part_fold(Part<SPLIT>& x, uint64_t& lo, uint64_t& hi) {
  uint64_t a = x.s1, ca = 0;
  if constexpr (SPLIT) {
    a += x.s1b;
    ca = a < x.s1b ? 1 : 0;
    x.s1b = 0;
  }
  const uint64_t t1 = a << 30, t2 = x.s2 << 60;
  uint64_t flo = x.s0 + t1;
  uint64_t fhi = (a >> 34) + (x.s2 >> 4) + (ca << 30) + (flo < t1 ? 1 : 0);
  flo += t2;
  fhi += flo < t2 ? 1 : 0;
  lo += flo;
  hi += fhi + (lo < flo ? 1 : 0);
  x.s0 = x.s1 = x.s2 = 0;
}

// Fold all 8 partial sums into their LDS totals; at fold f of each period of
// mac_chunk folds, total f (if any) is also Barrett-reduced.
template <bool SPLIT>
__device__ __forceinline__ void fold_lds(Part<SPLIT> (&acc)[8], u64x2* tot, uint32_t& nfold, uint32_t reduce_every,
                                         const LimbConst& lc) {
  const uint32_t f = nfold;
  nfold = f + 1 == reduce_every ? 0 : f + 1;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    u64x2 t = tot[i * kMacSlots];
    uint64_t lo = t[0], hi = t[1];
    part_fold(acc[i], lo, hi);
    if (f == (uint32_t)i) {
      lo = reduce128(hi, lo, lc.q, lc.mu_lo, lc.mu_hi);
      hi = 0;
    }
    tot[i * kMacSlots] = u64x2{lo, hi};
  }
}

// A wave-uniform 64-bit pointer, kept in scalar registers.
__device__ __forceinline__ const char* uni(const char* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const char*)(((uint64_t)hi << 32) | lo);
}

// Load at uniform base + per-lane byte offset (a scalar base and a 32-bit vector offset).
__device__ __forceinline__ uint64_t ld(const char* base, uint32_t off) {
  return *(const PENCIL_GLOBAL uint64_t*)((const PENCIL_GLOBAL char*)base + off);
}

// One term of a block's products: A rows and K columns advance through the
// contraction; the ciphertext side supplies both components (component 1 at
// c1 elements), the plaintext side one value for both.  Row and column
// pointers are wave-uniform (scalar registers); each lane adds its slot.
template <bool A_CT, bool SPLIT>
__device__ __forceinline__ void mac_term_v2(const MacTerm& T, const MacArgs& A, const Geo& G, const Consts& C,
                                            const LimbConst& lc, MacBlock& B, Part<SPLIT> (&acc)[8], u64x2* tot) {
  const int sp = G.nOY * G.nOX, kspan = G.nKY * G.nKX;
  const int ksteps = G.nK * kspan;
  const int64_t sa_str = (A_CT ? B.ct_stride : B.pt_stride) * 8, sk_str = (A_CT ? B.pt_stride : B.ct_stride) * 8;
  const int64_t c1 = T.c1 * 8;
  const uint32_t lane = (uint32_t)B.s * 8;
  const char* pa[2];
  const char* pk[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    int row = B.row0 + B.rg + a;
    if (row >= A.m_rows) row = B.row0 + B.rg;  // a padding row reads row 0 (never stored)
    const int mi = row / sp, rsp = row % sp;
    pa[a] = uni((const char*)(T.a + B.ln) + (((int64_t)mi * G.nK * sp + rsp) * kspan) * sa_str);
  }
#pragma unroll
  for (int c2 = 0; c2 < 2; ++c2) {
    int col = B.col0 + B.cg + c2;
    if (col >= G.nR) col = B.col0 + B.cg;
    pk[c2] = uni((const char*)(T.k + B.ln) + (int64_t)col * ksteps * sk_str);
  }
  const int64_t a_wrap = ((int64_t)(sp - 1) * kspan + 1) * sa_str;
  const uint32_t fold_every = SPLIT ? C.mac_fold4 : C.mac_fold, reduce_every = C.mac_chunk;
  int kk = 0, left = ksteps;
  struct Ops {
    uint64_t ct[2][2], pt[2];
  };
  auto load = [&](Ops& o) {
    // a copy of the lane offset made in this step, so that the loads below see
    // its zero-extension and take the scalar-base form (one register move
    // instead of a 64-bit address add per load)
    uint32_t off = lane;
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (A_CT) {
        o.ct[i][0] = ld(pa[i], off);
        o.ct[i][1] = ld(pa[i] + c1, off);
        o.pt[i] = ld(pk[i], off);
      } else {
        o.pt[i] = ld(pa[i], off);
        o.ct[i][0] = ld(pk[i], off);
        o.ct[i][1] = ld(pk[i] + c1, off);
      }
    }
    const bool adv = --left > 0;
    const int64_t da = !adv ? 0 : (kk + 1 == kspan) ? a_wrap : sa_str;
    const int64_t dk = adv ? sk_str : 0;
    kk = (kk + 1 == kspan) ? 0 : kk + 1;
    pa[0] = uni(pa[0] + da);
    pa[1] = uni(pa[1] + da);
    pk[0] = uni(pk[0] + dk);
    pk[1] = uni(pk[1] + dk);
  };
  auto step = [&](const Ops& o) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const uint64_t av = A_CT ? o.ct[a][c] : o.pt[a];
          const uint64_t kv = A_CT ? o.pt[c2] : o.ct[c2][c];
          part_mac(acc[(a * 2 + c2) * 2 + c], av, kv);
        }
    if (++B.nmac == fold_every) {
      B.nmac = 0;
      fold_lds(acc, tot, B.nfold, reduce_every, lc);
    }
  };
  Ops x, y, z;
  load(x);
  load(y);
  for (int k = 0; k < ksteps; k += 3) {
    load(z);
    step(x);
    if (k + 1 >= ksteps) break;
    load(x);
    step(y);
    if (k + 2 >= ksteps) break;
    load(y);
    step(z);
  }
}

template <int ROWS, int COLS, bool SPLIT>
__device__ __forceinline__ void do_mac_v2(u64x2* lds, const MacArgs& A, const Geo& G, const Consts& C,
                                          int slot_block, int chunk) {
  constexpr int WC = COLS / 2;
  static_assert((ROWS / 2) * WC == 8, "8 waves per block");
  const int n = C.n, L = C.L;
  const int per_limb = n / kMacSlots;
  const int l = slot_block / per_limb;
  const LimbConst& lc = C.limb[l];
  const int cchunks = (G.nR + COLS - 1) / COLS;
  MacBlock B;
  B.row0 = (chunk / cchunks) * ROWS;
  B.col0 = (chunk % cchunks) * COLS;
  B.s = threadIdx.x & (kMacSlots - 1);
  B.grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  B.comp = 0;
  B.rg = (B.grp / WC) * 2;
  B.cg = (B.grp % WC) * 2;
  B.ln = (int64_t)l * n + (int64_t)(slot_block % per_limb) * kMacSlots;
  B.ct_stride = 2 * (int64_t)L * n;
  B.pt_stride = (int64_t)L * n;
  B.active = B.row0 + B.rg < A.m_rows && B.col0 + B.cg < G.nR;
  B.nmac = B.nfold = 0;
  if (!B.active) return;
  u64x2* tot = lds + B.grp * 8 * kMacSlots + B.s;  // this lane's 8 totals, stride kMacSlots
#pragma unroll
  for (int i = 0; i < 8; ++i) tot[i * kMacSlots] = u64x2{0, 0};
  Part<SPLIT> acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = Part<SPLIT>{};
  // term 0 has the ciphertext on the A side (forward, input gradient, the
  // weight gradient's term A); the weight gradient's term B has it on the K side
  mac_term_v2<true, SPLIT>(A.term[0], A, G, C, lc, B, acc, tot);
  if (A.n_terms > 1) mac_term_v2<false, SPLIT>(A.term[1], A, G, C, lc, B, acc, tot);
  // re-randomisation term pk_c * u'_o, reduction and store
  const int64_t ln = B.ln, pt_stride = B.pt_stride, ct_stride = B.ct_stride;
  const int s = B.s, sp = G.nOY * G.nOX;
  const PENCIL_GLOBAL uint64_t* gpk = gview(A.pk);
  const PENCIL_GLOBAL uint64_t* gu = gview(A.u);
  PENCIL_GLOBAL uint64_t* gout = gview(A.out);
  const uint64_t pk0 = gpk[ln + s], pk1 = gpk[pt_stride + ln + s];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int row = B.row0 + B.rg + a;
    if (row >= A.m_rows) continue;
    const int mi = row / sp, oyi = (row % sp) / G.nOX, oxi = row % G.nOX;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = B.col0 + B.cg + b;
      if (col >= G.nR) continue;
      const int64_t o = (((int64_t)mi * G.nR + col) * G.nOY + oyi) * G.nOX + oxi;
      const uint64_t u = gu[o * pt_stride + ln + s];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int i = (a * 2 + b) * 2 + c;
        Part<SPLIT>& x = acc[i];
        part_mac(x, c ? pk1 : pk0, u);  // one more step: the partial sums hold fewer than a fold's steps
        const u64x2 t = tot[i * kMacSlots];
        uint64_t lo = t[0], hi = t[1];
        part_fold(x, lo, hi);
        gout[o * ct_stride + (int64_t)c * pt_stride + ln + s] = reduce128(hi, lo, lc.q, lc.mu_lo, lc.mu_hi);
      }
    }
  }
}

constexpr int kMacV2Lds = 8 * 8 * kMacSlots;  // u64x2 words: 8 waves x 8 totals x 64 lanes (64 KiB)

// Kind 0: LDS-staged 2 x 2 wave blocks, both components; 2: direct 2 x 2
// wave blocks of one component each (kind 1 is do_mac_kind1).
template <int KIND>
__device__ __forceinline__ void do_mac(uint64_t* smem, const MacArgs& A, const Geo& G, const Consts& C,
                                       int slot_block, int chunk) {
  constexpr bool DIRECT = KIND != 0;
  constexpr int NC = KIND == 2 ? 1 : 2;
  switch (A.variant % 3) {
    case 1: do_mac_t<2, KIND == 2 ? 8 : 16, 2, 2, NC, DIRECT>(smem, A, G, C, slot_block, chunk); break;
    case 2: do_mac_t<8, KIND == 2 ? 2 : 4, 2, 2, NC, DIRECT>(smem, A, G, C, slot_block, chunk); break;
    default: do_mac_t<4, KIND == 2 ? 4 : 8, 2, 2, NC, DIRECT>(smem, A, G, C, slot_block, chunk); break;
  }
}

// Work item of block `b` of `total`.  Workgroups go to the 8 XCDs round-robin
// by block index, so XCD x = b mod 8 receives blocks b = x, x + 8, ...; giving
// it the contiguous work range [x total / 8, (x + 1) total / 8) in order keeps
// the chunks of one slot range (which share operands) on one L2.
__global__ void __launch_bounds__(512) k_mac_lds(MacArgs A, Geo G, Consts C, int chunks, int64_t total) {
  extern __shared__ uint64_t smem[];
  const int w = (int)xcd_work(blockIdx.x, total);
  do_mac<0>(smem, A, G, C, w / chunks, w % chunks);
}

// Kind 1 through do_mac_v2: 2 x 2 wave blocks, both components, totals in LDS.
template <bool SPLIT>
__device__ __forceinline__ void do_mac_kind1(u64x2* tot, const MacArgs& A, const Geo& G, const Consts& C, int w,
                                             int chunks) {
  switch (A.variant % 3) {
    case 1: do_mac_v2<2, 16, SPLIT>(tot, A, G, C, w / chunks, w % chunks); break;
    case 2: do_mac_v2<8, 4, SPLIT>(tot, A, G, C, w / chunks, w % chunks); break;
    default: do_mac_v2<4, 8, SPLIT>(tot, A, G, C, w / chunks, w % chunks); break;
  }
}

__global__ void __launch_bounds__(512) k_mac_direct(MacArgs A, Geo G, Consts C, int chunks, int64_t total) {
  __shared__ u64x2 tot[kMacV2Lds];
  const int w = (int)xcd_work(blockIdx.x, total);
  do_mac_kind1<false>(tot, A, G, C, w, chunks);
}

__global__ void __launch_bounds__(512) k_mac_direct_small(MacArgs A, Geo G, Consts C, int chunks, int64_t total) {
  const int w = (int)xcd_work(blockIdx.x, total);
  do_mac<2>(nullptr, A, G, C, w / chunks, w % chunks);
}

// Every multiply-accumulate of one step with one staging kind.  Segments start
// at multiples of 8 blocks, so a segment's blocks keep their XCD under the
// per-segment work remap; padding blocks past the segment's work exit.
template <int KIND>
__device__ __forceinline__ void step_mac(const StepSeg* __restrict__ segs, int nseg,
                                         const Consts* __restrict__ consts, uint64_t* smem) {
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const int64_t local = (int64_t)blockIdx.x - S.block_begin;
  const int chunks = mac_chunks(S.mac.variant, S.mac.m_rows, S.G.nR);
  const int64_t work = S.slot_blocks * chunks, padded = (work + 7) & ~(int64_t)7;
  const int w = (int)xcd_work(local, padded);  // work items per launch stay below 2^31
  if (w >= work) return;
  do_mac<KIND>(smem, S.mac, S.G, consts[S.ctx], w / chunks, w % chunks);
}

#define STEP_ARGS const StepSeg *__restrict__ segs, int nseg, const Consts *__restrict__ consts
__global__ void __launch_bounds__(512) k_step_mac(STEP_ARGS) {
  __shared__ uint64_t smem[kMacSmemWords];
  step_mac<0>(segs, nseg, consts, smem);
}

__global__ void __launch_bounds__(512, 4) k_step_mac_direct(STEP_ARGS) {
  __shared__ u64x2 tot[kMacV2Lds];
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const int64_t local = (int64_t)blockIdx.x - S.block_begin;
  const int chunks = mac_chunks(S.mac.variant, S.mac.m_rows, S.G.nR);
  const int64_t work = S.slot_blocks * chunks, padded = (work + 7) & ~(int64_t)7;
  const int w = (int)xcd_work(local, padded);  // work items per launch stay below 2^31
  if (w >= work) return;
  do_mac_kind1<true>(tot, S.mac, S.G, consts[S.ctx], w, chunks);
}

__global__ void __launch_bounds__(512) k_step_mac_direct_small(STEP_ARGS) {
  step_mac<2>(segs, nseg, consts, nullptr);
}
#undef STEP_ARGS

hipError_t launch_mac(const MacArgs& A, int64_t n_out, const Geo& G, const Consts& C, hipStream_t s) {
  if (n_out <= 0) return hipSuccess;
  // the kernels take term 0 with the ciphertext on the A side and an optional
  // term 1 with it on the K side
  if (A.n_terms < 1 || A.n_terms > 2 || !A.term[0].a_is_ct || (A.n_terms == 2 && A.term[1].a_is_ct))
    return hipErrorInvalidValue;
  const int64_t slot_blocks = (int64_t)C.n * C.L / kMacSlots;
  const int chunks = mac_chunks(A.variant, A.m_rows, G.nR);
  const int64_t total = slot_blocks * chunks;
  if (total >= (1ll << 31)) return hipErrorInvalidConfiguration;  // work items are int
  if (A.variant >= 6)
    hipLaunchKernelGGL(k_mac_direct_small, dim3((unsigned)total), dim3(512), 0, s, A, G, C, chunks, total);
  else if (A.variant >= 3)
    hipLaunchKernelGGL(k_mac_direct, dim3((unsigned)total), dim3(512), 0, s, A, G, C, chunks, total);
  else
    hipLaunchKernelGGL(k_mac_lds, dim3((unsigned)total), dim3(512), kMacSmemWords * sizeof(uint64_t), s, A, G, C,
                       chunks, total);
  return hipGetLastError();
}

hipError_t launch_step_mac(const StepPhase& P, int64_t blocks, int kind, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (kind == 2)
    hipLaunchKernelGGL(k_step_mac_direct_small, dim3((unsigned)blocks), dim3(512), 0, s, P.segs, P.nseg, P.consts);
  else if (kind == 1)
    hipLaunchKernelGGL(k_step_mac_direct, dim3((unsigned)blocks), dim3(512), 0, s, P.segs, P.nseg, P.consts);
  else
    hipLaunchKernelGGL(k_step_mac, dim3((unsigned)blocks), dim3(512), 0, s, P.segs, P.nseg, P.consts);
  return hipGetLastError();
}

hipError_t configure_lds_mac() {
  const int mac_lds = kMacSmemWords * sizeof(uint64_t);
  hipError_t m1 = hipFuncSetAttribute((const void*)k_mac_lds, hipFuncAttributeMaxDynamicSharedMemorySize, mac_lds);
  hipError_t m2 = hipFuncSetAttribute((const void*)k_step_mac, hipFuncAttributeMaxDynamicSharedMemorySize, mac_lds);
  return m1 != hipSuccess ? m1 : m2;
}

}  // namespace pencil
