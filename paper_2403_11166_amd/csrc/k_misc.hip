// Flood and mask of the products' outputs, the Z_t kernels (local terms,
// Pencil+ online correlations and combinations), the bias gradient, the DP
// perturbation, stride relayouts and the step's nonce counter.
#include <mutex>

#include "device_common.h"

namespace pencil {


// Output ciphertexts after the inverse NTT: c0 += e0' + flood - round(q s / t),
// c1 += e1'; the model owner's share is s at the output slots (+ bias).
// Each thread handles 4 consecutive coefficients of one output ciphertext.
template <int W>
__device__ __forceinline__ void do_flood(uint64_t* ct, int64_t n_out, int64_t* share0, const int64_t* bias,
                                         const Geo& G, const View& OV, uint64_t nonce, uint64_t obj_base,
                                         const Consts& C, int64_t g) {
  const int n = C.n, L = C.L;
  const int per_log = C.log2n - 2;  // a thread takes 4 of the N coefficients of one output
  if (g >= (n_out << per_log)) return;
  const int64_t o = g >> per_log;
  const int n0 = (int)(g & ((1 << per_log) - 1)) * 4;
  const uint64_t obj = obj_base + (uint64_t)o;
  const uint64_t blk4 = (uint64_t)(n0 / 4);
  U64x4 e0 = philox(blk4, obj, P_RR_E0, 0, C.seed, nonce);
  U64x4 e1 = philox(blk4, obj, P_RR_E1, 0, C.seed, nonce);
  U64x4 mk0 = philox(2 * blk4, obj, P_MASK, 0, C.seed, nonce);
  U64x4 mk1 = philox(2 * blk4 + 1, obj, P_MASK, 0, C.seed, nonce);
  uint64_t fw[4 * W];  // the 4W flood words of these 4 coefficients, in stream order
#pragma unroll
  for (int b = 0; b < W; ++b) {
    U64x4 f = philox(blk4 * W + b, obj, P_FLOOD, 0, C.seed, nonce);
#pragma unroll
    for (int z = 0; z < 4; ++z) fw[b * 4 + z] = f.v[z];
  }
  const int64_t ct_stride = 2 * (int64_t)L * n;
  PENCIL_GLOBAL uint64_t* c0p = gview(ct) + o * ct_stride;
  PENCIL_GLOBAL uint64_t* c1p = c0p + (int64_t)L * n;
  // output-tile coordinates of o = ((mi*nR + ri)*nOY + oyi)*nOX + oxi, in
  // 32-bit arithmetic (a step's outputs number far fewer than 2^32)
  uint32_t ti = (uint32_t)o;
  const int oxi = (int)(ti % (uint32_t)G.nOX);
  ti /= (uint32_t)G.nOX;
  const int oyi = (int)(ti % (uint32_t)G.nOY);
  ti /= (uint32_t)G.nOY;
  const int ri = (int)(ti % (uint32_t)G.nR);
  const int mi = (int)(ti / (uint32_t)G.nR);
  // per-coefficient draws: re-randomisation errors, the mask s = (wlo + 2^64 whi) mod t
  int64_t ev0[4], ev1[4];
  uint64_t sv[4], rrv[4];
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    ev0[z] = cbd21(e0.v[z]);
    ev1[z] = cbd21(e1.v[z]);
    const uint64_t wlo = (z < 2 ? mk0 : mk1).v[(2 * z) & 3], whi = (z < 2 ? mk0 : mk1).v[(2 * z + 1) & 3];
    uint64_t sh = reduce64(whi, C.one_sh_t, C.t);
    uint64_t sz = mul_shoup(sh, C.r64t, C.r64t_sh, C.t) + reduce64(wlo, C.one_sh_t, C.t);
    if (sz >= C.t) sz -= C.t;
    sv[z] = sz;
    rrv[z] = round_rho(sz, C);
  }
  // the thread's 4 consecutive coefficients of each limb move as two 16-byte words
  for (int l = 0; l < L; ++l) {
    const LimbConst& lc = C.limb[l];
    PENCIL_GLOBAL u64x2* p0 = (PENCIL_GLOBAL u64x2*)(c0p + (int64_t)l * n + n0);
    PENCIL_GLOBAL u64x2* p1 = (PENCIL_GLOBAL u64x2*)(c1p + (int64_t)l * n + n0);
    const u64x2 a0 = p0[0], a1 = p0[1], b0 = p1[0], b1 = p1[1];
    uint64_t x0[4] = {a0.x, a0.y, a1.x, a1.y}, x1[4] = {b0.x, b0.y, b1.x, b1.y};
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      // flood value V - 2^fb with V = sum_b w_b 2^(64 b) the low fb+1 bits of the
      // words: sum_b w_b (2^(64 b) mod q) < 2^126 as one 128-bit value, one reduction
      uint64_t hi = 0, lo = fw[z * W];
#pragma unroll
      for (int b = 1; b < W; ++b) {
        uint64_t w = fw[z * W + b];
        if (b == W - 1) w &= C.top_mask;
        uint64_t ph, pl;
        mul_wide(w, b == 1 ? lc.r64 : b == 2 ? lc.r128 : lc.r192, ph, pl);
        lo += pl;
        hi += ph + (lo < pl ? 1 : 0);
      }
      if (W == 1) lo &= C.top_mask;
      uint64_t v = reduce128(hi, lo, lc.q, lc.mu_lo, lc.mu_hi);
      v = sub_mod(v, lc.flood_off, lc.q);
      uint64_t c = add_mod(x0[z], small_to_mod(ev0[z], lc.q), lc.q);
      c = add_mod(c, v, lc.q);
      x0[z] = sub_mod(c, delta_scale(sv[z], rrv[z], lc), lc.q);
      x1[z] = add_mod(x1[z], small_to_mod(ev1[z], lc.q), lc.q);
    }
    p0[0] = u64x2{x0[0], x0[1]};
    p0[1] = u64x2{x0[2], x0[3]};
    p1[0] = u64x2{x1[0], x1[1]};
    p1[1] = u64x2{x1[2], x1[3]};
  }
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    const int i = n0 + z;
    const uint64_t s = sv[z];
    // model owner's share at the output slots: slot = mm*RS + O + rr*S + y*wa + x
    int zz = i - G.O;
    if (zz >= 0) {
      const int mm = fdiv(zz, G.dv_rs);
      const int rem = zz - mm * G.RS;
      const int rr2 = fdiv(rem, G.dv_s);
      const int rem2 = rem - rr2 * G.S;
      const int y = fdiv(rem2, G.dv_wa), x = rem2 - y * G.wa;
      if (mm < G.mt && y < G.oh && x < G.ow) {
        int m = mi * G.mt + mm, r = ri * G.rt + rr2, yy = oyi * G.oh + y, xx = oxi * G.ow + x;
        if (m < G.M && r < G.R && yy < G.OH && xx < G.OW) {
          uint64_t val = s;
          if (bias) {
            val += (uint64_t)gview(bias)[r];
            if (val >= C.t) val -= C.t;
          }
          gview(share0)[m * OV.s0 + r * OV.s1 + yy * OV.sy + xx * OV.sx] = (int64_t)val;
        }
      }
    }
  }
}

template <int W>
__global__ void __launch_bounds__(256) k_flood_mask(uint64_t* ct, int64_t n_out, int64_t* share0,
                                                    const int64_t* bias, Geo G, View OV, uint64_t nonce,
                                                    uint64_t obj_base, Consts C) {
  do_flood<W>(ct, n_out, share0, bias, G, OV, nonce, obj_base, C, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Exact Z_t packed correlation of two plaintext tensors, one thread per output
// element: out[m, r, y, x] = sum_{k, dy, dx} A[m, k, y+dy, x+dx] K[r, k, dy, dx]
// mod t, with 128-bit accumulation (41-bit operands, < 2^46 terms).  Used for
// the local terms of the weight gradient.
__global__ void __launch_bounds__(256) k_zt_corr(const int64_t* a, const int64_t* kt, int64_t* out, Geo G, View AV,
                                                 View KV, View OV, Consts C) {
  const int64_t total = (int64_t)G.M * G.R * G.OH * G.OW;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int64_t e = g;
  const int x = (int)(e % G.OW);
  e /= G.OW;
  const int y = (int)(e % G.OH);
  e /= G.OH;
  const int r = (int)(e % G.R);
  const int m = (int)(e / G.R);
  uint64_t hi = 0, lo = 0;
  for (int k = 0; k < G.K; ++k)
    for (int dy = 0; dy < G.KH; ++dy) {
      const int ys = y + dy - AV.pady;
      if (ys < 0 || ys >= AV.H) continue;
      for (int dx = 0; dx < G.KW; ++dx) {
        const int xs = x + dx - AV.pad;
        if (xs < 0 || xs >= AV.W) continue;
        const uint64_t av = (uint64_t)a[m * AV.s0 + k * AV.s1 + ys * AV.sy + xs * AV.sx];
        const int ky = KV.flip ? KV.KH - 1 - dy : dy, kx = KV.flip ? KV.KW - 1 - dx : dx;
        const uint64_t kv = (uint64_t)kt[r * KV.s0 + k * KV.s1 + ky * KV.sy + kx * KV.sx];
        uint64_t ph, pl;
        mul_wide(av, kv, ph, pl);
        lo += pl;
        hi += ph + (lo < pl ? 1 : 0);
      }
    }
  // (hi 2^64 + lo) mod t
  uint64_t v = add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t),
                       reduce64(lo, C.one_sh_t, C.t), C.t);
  out[m * OV.s0 + r * OV.s1 + y * OV.sy + x * OV.sx] = (int64_t)v;
}

// The same correlation as a tiled contraction.  A workgroup of nw waves owns a
// (8 TI) x (8 TI) tile of (output position, output channel) pairs, each lane a
// TI x TI block, and the waves split the contraction (k, dy, dx) nw ways.
// Operands (< t < 2^42) are split into 21-bit halves, so a product is four
// 32 x 32 multiply-adds into three 64-bit partial sums that hold 2^22 terms;
// each wave reduces its totals mod t and the waves' results are summed through
// LDS.  The launcher picks TI and nw so that small outputs or short
// contractions still fill the GPU.
constexpr int kZtWaves = 16;
template <int TI>
__global__ void __launch_bounds__(1024) k_zt_gemm(const int64_t* a, const int64_t* kt, int64_t* out, Geo G, View AV,
                                                  View KV, View OV, Consts C) {
  constexpr int NO = 64 * TI * TI;  // outputs per workgroup
  __shared__ uint64_t red[kZtWaves][NO];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int P = G.M * G.OH * G.OW, R = G.R, ohw = G.OH * G.OW;
  const PENCIL_GLOBAL int64_t* ga = gview(a);
  const PENCIL_GLOBAL int64_t* gk = gview(kt);
  int64_t abase[TI];
  int ay[TI], ax[TI];
  bool rv[TI];
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const int row = blockIdx.x * 8 * TI + (lane >> 3) * TI + i;
    rv[i] = row < P;
    const int rr = rv[i] ? row : 0;
    const int m = rr / ohw, rem = rr - m * ohw, y = rem / G.OW, x = rem - y * G.OW;
    abase[i] = (int64_t)m * AV.s0;
    ay[i] = y - AV.pady;
    ax[i] = x - AV.pad;
  }
  int64_t kbase[TI];
  bool cv[TI];
#pragma unroll
  for (int j = 0; j < TI; ++j) {
    const int col = blockIdx.y * 8 * TI + (lane & 7) * TI + j;
    cv[j] = col < R;
    kbase[j] = (int64_t)(cv[j] ? col : 0) * KV.s0;
  }
  const int kk = G.KH * G.KW;
  const int64_t ctot = (int64_t)G.K * kk, per = (ctot + nw - 1) / nw;
  const int64_t c_begin = wv * per, c_end = c_begin + per < ctot ? c_begin + per : ctot;
  uint64_t s0[TI][TI] = {}, s1[TI][TI] = {}, s2[TI][TI] = {};
  int k = 0, dy = 0, dx = 0;
  if (c_begin < c_end) {
    k = (int)(c_begin / kk);
    const int rem = (int)(c_begin - (int64_t)k * kk);
    dy = rem / G.KW;
    dx = rem - dy * G.KW;
  }
  constexpr uint64_t kLo = (1ull << 21) - 1;
  // Chunks of U contraction steps: all loads of a chunk are issued before its
  // multiply-adds.
  constexpr int U = 4;
  for (int64_t c0 = c_begin; c0 < c_end; c0 += U) {
    uint64_t av[U][TI], bv[U][TI];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool live = c0 + u < c_end;
      const int ky = KV.flip ? KV.KH - 1 - dy : dy, kx = KV.flip ? KV.KW - 1 - dx : dx;
      const int64_t koff = (int64_t)k * KV.s1 + (int64_t)ky * KV.sy + (int64_t)kx * KV.sx;
#pragma unroll
      for (int j = 0; j < TI; ++j) bv[u][j] = live && cv[j] ? (uint64_t)gk[kbase[j] + koff] : 0;
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const int ys = ay[i] + dy, xs = ax[i] + dx;
        const bool in = live && rv[i] && ys >= 0 && ys < AV.H && xs >= 0 && xs < AV.W;
        av[u][i] = in ? (uint64_t)ga[abase[i] + (int64_t)k * AV.s1 + (int64_t)ys * AV.sy + (int64_t)xs * AV.sx] : 0;
      }
      if (++dx == G.KW) {
        dx = 0;
        if (++dy == G.KH) {
          dy = 0;
          ++k;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const uint32_t a0 = (uint32_t)(av[u][i] & kLo), a1 = (uint32_t)(av[u][i] >> 21);
#pragma unroll
        for (int j = 0; j < TI; ++j) {
          const uint32_t b0 = (uint32_t)(bv[u][j] & kLo), b1 = (uint32_t)(bv[u][j] >> 21);
          s0[i][j] += (uint64_t)a0 * b0;
          s1[i][j] += (uint64_t)a0 * b1;
          s1[i][j] += (uint64_t)a1 * b0;
          s2[i][j] += (uint64_t)a1 * b1;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TI; ++j) {
      // s0 + s1 2^21 + s2 2^42 as a 128-bit value, then mod t
      const uint64_t t1 = s1[i][j] << 21, t2 = s2[i][j] << 42;
      uint64_t lo = s0[i][j] + t1;
      uint64_t hi = (lo < t1 ? 1 : 0) + (s1[i][j] >> 43) + (s2[i][j] >> 22);
      lo += t2;
      hi += lo < t2 ? 1 : 0;
      red[wv][(lane * TI + i) * TI + j] = add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t),
                                                  reduce64(lo, C.one_sh_t, C.t), C.t);
    }
  __syncthreads();
  for (int o = threadIdx.x; o < NO; o += blockDim.x) {
    const int ol = o / (TI * TI), i = (o / TI) % TI, j = o % TI;
    uint64_t v = 0;
    for (int w = 0; w < nw; ++w) v = add_mod(v, red[w][o], C.t);
    const int row = blockIdx.x * 8 * TI + (ol >> 3) * TI + i, col = blockIdx.y * 8 * TI + (ol & 7) * TI + j;
    if (row < P && col < R) {
      const int m = row / ohw, rem = row - m * ohw, y = rem / G.OW, x = rem - y * G.OW;
      gview(out)[(int64_t)m * OV.s0 + (int64_t)col * OV.s1 + (int64_t)y * OV.sy + (int64_t)x * OV.sx] = (int64_t)v;
    }
  }
}

// The same correlation on the fp64 matrix cores.  Each operand, centred into
// (-t/2, t/2), is split into DIG signed digits of B = 21 (DIG = 2) or 14
// (DIG = 3) bits, v = d0 + d1 2^B [+ d2 2^2B] (all but the top digit in
// [0, 2^B), the top one the signed rest); the DIG^2 digit products of a pair
// land on 2 DIG - 1 diagonals T_s = sum d_i e_j (i + j = s), each a
// 16 x 16 x 4 fp64 multiply-accumulate.  Every digit product and running sum
// is an integer below 2^53 (the launcher bounds the terms per wave, and takes
// two digits only while t < 2^42), so the fp64 arithmetic is exact; at the end
// each T_s is reduced mod t and the diagonals are recombined with 2^(B s) mod
// t.  A workgroup owns a 16 x 16 output tile and splits the contraction over
// its waves, four contraction indices per step.  Lane l holds
// A[row l % 16][c + l / 16] and B[c + l / 16][col l % 16], and register r of
// its accumulator holds output (l / 16 + 4 r, l % 16).
typedef double zt_v4d __attribute__((ext_vector_type(4)));

template <int DIG>
__device__ __forceinline__ void zt_digits(uint64_t v, const Consts& C, double (&d)[DIG]) {
  constexpr int B = DIG == 2 ? 21 : 14;
  int64_t c = v > C.t_half ? (int64_t)v - (int64_t)C.t : (int64_t)v;
#pragma unroll
  for (int i = 0; i < DIG - 1; ++i) {
    d[i] = (double)(c & ((1ll << B) - 1));
    c >>= B;
  }
  d[DIG - 1] = (double)c;
}

__device__ __forceinline__ uint64_t zt_mod_signed(int64_t x, const Consts& C) {
  const uint64_t u = x < 0 ? (uint64_t)(-x) : (uint64_t)x;
  const uint64_t r = reduce64(u, C.one_sh_t, C.t);
  return x < 0 && r ? C.t - r : r;
}

template <int DIG>
__global__ void __launch_bounds__(1024) k_zt_mfma(const int64_t* a, const int64_t* kt, int64_t* out, Geo G, View AV,
                                                  View KV, View OV, Consts C) {
  __shared__ uint64_t red[kZtWaves][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int P = G.M * G.OH * G.OW, R = G.R, ohw = G.OH * G.OW;
  const PENCIL_GLOBAL int64_t* ga = gview(a);
  const PENCIL_GLOBAL int64_t* gk = gview(kt);
  const int lr = lane & 15, lc = lane >> 4;
  // this lane's A row and B column
  const int row = blockIdx.x * 16 + lr, col = blockIdx.y * 16 + lr;
  const bool rv = row < P, cv = col < R;
  int64_t abase, kbase;
  int ay, ax;
  {
    const int rr = rv ? row : 0;
    const int m = rr / ohw, rem = rr - m * ohw, y = rem / G.OW, x = rem - y * G.OW;
    abase = (int64_t)m * AV.s0;
    ay = y - AV.pady;
    ax = x - AV.pad;
    kbase = (int64_t)(cv ? col : 0) * KV.s0;
  }
  const int kk = G.KH * G.KW;
  const int64_t ctot = (int64_t)G.K * kk;
  const int64_t steps = (ctot + 3) / 4, per = (steps + nw - 1) / nw;
  const int64_t s_begin = wv * per, s_end = s_begin + per < steps ? s_begin + per : steps;
  constexpr int ND = 2 * DIG - 1, B = DIG == 2 ? 21 : 14;
  zt_v4d acc[ND];
#pragma unroll
  for (int s = 0; s < ND; ++s) acc[s] = zt_v4d{0, 0, 0, 0};
  // this lane's contraction index c = 4 step + lc as (k, dy, dx), divided out
  // once and then advanced by 4 per step
  int k = 0, dy = 0, dx = 0;
  {
    const int64_t c = s_begin * 4 + lc;
    k = (int)(c / kk);
    const int rem = (int)(c - (int64_t)k * kk);
    dy = rem / G.KW;
    dx = rem - dy * G.KW;
  }
  constexpr int U = 4;  // contraction steps whose loads are issued together
  for (int64_t st0 = s_begin; st0 < s_end; st0 += U) {
    uint64_t av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = (st0 + u) * 4 + lc;
      const bool live = st0 + u < s_end && c < ctot;
      const int ky = KV.flip ? KV.KH - 1 - dy : dy, kx = KV.flip ? KV.KW - 1 - dx : dx;
      bv[u] = live && cv ? (uint64_t)gk[kbase + (int64_t)k * KV.s1 + (int64_t)ky * KV.sy + (int64_t)kx * KV.sx] : 0;
      const int ys = ay + dy, xs = ax + dx;
      const bool in = live && rv && ys >= 0 && ys < AV.H && xs >= 0 && xs < AV.W;
      av[u] = in ? (uint64_t)ga[abase + (int64_t)k * AV.s1 + (int64_t)ys * AV.sy + (int64_t)xs * AV.sx] : 0;
      if (kk == 1) {
        k += 4;
      } else {
        dx += 4;
        while (dx >= G.KW) {
          dx -= G.KW;
          if (++dy == G.KH) {
            dy = 0;
            ++k;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double da[DIG], db[DIG];
      zt_digits<DIG>(av[u], C, da);
      zt_digits<DIG>(bv[u], C, db);
#pragma unroll
      for (int i = 0; i < DIG; ++i)
#pragma unroll
        for (int j = 0; j < DIG; ++j)
          acc[i + j] = __builtin_amdgcn_mfma_f64_16x16x4f64(da[i], db[j], acc[i + j], 0, 0, 0);
    }
  }
  // 2^(B s) mod t
  uint64_t pw[ND];
  pw[0] = 1;
#pragma unroll
  for (int s = 1; s < ND; ++s) pw[s] = reduce64((uint64_t)1 << (B * s), C.one_sh_t, C.t);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    uint64_t hi = 0, lo = 0;
#pragma unroll
    for (int s = 0; s < ND; ++s) {
      uint64_t ph, pl;
      mul_wide(zt_mod_signed((int64_t)acc[s][r], C), pw[s], ph, pl);
      lo += pl;
      hi += ph + (lo < pl ? 1 : 0);
    }
    red[wv][(lc + 4 * r) * 16 + lr] =
        add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t), reduce64(lo, C.one_sh_t, C.t), C.t);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 256; o += blockDim.x) {
    uint64_t v = 0;
    for (int w = 0; w < nw; ++w) v = add_mod(v, red[w][o], C.t);
    const int orow = blockIdx.x * 16 + o / 16, ocol = blockIdx.y * 16 + o % 16;
    if (orow < P && ocol < R) {
      const int m = orow / ohw, rem = orow - m * ohw, y = rem / G.OW, x = rem - y * G.OW;
      gview(out)[(int64_t)m * OV.s0 + (int64_t)ocol * OV.s1 + (int64_t)y * OV.sy + (int64_t)x * OV.sx] = (int64_t)v;
    }
  }
}

// The correlation for output grids too small to fill the GPU with tiles but
// with a long contraction (fully connected forward products, weight gradients
// of layers with few channels).  A wave owns a 2 x 2 block of (row, column)
// outputs and its 64 lanes split the contraction (lane l takes the flattened
// indices c = (k, dy, dx) with c = l mod 64 NWB); with NWB = 4 the four waves
// of a workgroup share one block and split it four ways, else a workgroup
// holds four blocks.  An operand stored contiguously along the contraction is
// read with coalesced loads.  Products use the 21-bit halves of the vector
// kernel; the partial sums of all lanes (and waves) of a block, which hold the
// whole contraction (the launcher bounds its length), are added by shuffles
// (and through LDS), and four lanes then reduce one output each.  A lane
// advances its index by the mixed-radix digits (D.dk, D.ddy, D.ddx) of the
// stride 64 NWB.  WIN = false is the fully connected form (1 x 1 kernel and
// output, no padding): the contraction index is the channel alone.
struct DotStep {
  int32_t dk, ddy, ddx, pad;
};

template <int NWB, bool WIN>
__global__ void __launch_bounds__(256) k_zt_dot(const int64_t* a, const int64_t* kt, int64_t* out, Geo G, View AV,
                                                View KV, View OV, Consts C, DotStep D) {
  __shared__ uint64_t red[4][4][3];  // NWB = 4: [wave][output][partial sum]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t blk = NWB == 1 ? (int64_t)blockIdx.x * 4 + wv : (int64_t)blockIdx.x;
  const int ohw = G.OH * G.OW, P = G.M * ohw, R = G.R, kk = G.KH * G.KW;
  const int cb = (R + 1) / 2;
  // the whole wave (NWB = 1) or workgroup (NWB = 4) leaves together
  if (blk >= (int64_t)((P + 1) / 2) * cb) return;
  const int row0 = (int)(blk / cb) * 2, col0 = (int)(blk % cb) * 2;
  const PENCIL_GLOBAL int64_t* ga = gview(a);
  const PENCIL_GLOBAL int64_t* gk = gview(kt);
  int64_t abase[2], kbase[2];
  int ay[2], ax[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = row0 + i < P ? row0 + i : row0;  // a padding row repeats row0 (never stored)
    const int m = WIN ? row / ohw : row, rem = row - m * ohw, y = WIN ? rem / G.OW : 0, x = rem - y * G.OW;
    abase[i] = (int64_t)m * AV.s0;
    ay[i] = y - AV.pady;
    ax[i] = x - AV.pad;
    const int col = col0 + i < R ? col0 + i : col0;
    kbase[i] = (int64_t)col * KV.s0;
  }
  const int ctot = G.K * kk;  // at most 2^22 (the launcher's bound)
  const int stride = 64 * NWB;
  int c = lane + 64 * (NWB == 1 ? 0 : wv);
  int k = c, dy = 0, dx = 0;
  if constexpr (WIN) {
    k = c / kk;
    const int rem = c - k * kk;
    dy = rem / G.KW;
    dx = rem - dy * G.KW;
  }
  constexpr uint64_t kLo = (1ull << 21) - 1;
  uint64_t s0[4] = {}, s1[4] = {}, s2[4] = {};
  constexpr int U = 4;  // contraction indices per lane whose loads are issued together
  for (; c < ctot; c += stride * U) {
    uint64_t av[U][2], bv[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool live = c + stride * u < ctot;
      if constexpr (!WIN) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          av[u][i] = live ? (uint64_t)ga[abase[i] + (int64_t)k * AV.s1] : 0;
          bv[u][i] = live ? (uint64_t)gk[kbase[i] + (int64_t)k * KV.s1] : 0;
        }
        k += stride;
        continue;
      }
      const int ky = KV.flip ? KV.KH - 1 - dy : dy, kx = KV.flip ? KV.KW - 1 - dx : dx;
      const int64_t koff = (int64_t)k * KV.s1 + (int64_t)ky * KV.sy + (int64_t)kx * KV.sx;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int ys = ay[i] + dy, xs = ax[i] + dx;
        const bool in = live && ys >= 0 && ys < AV.H && xs >= 0 && xs < AV.W;
        av[u][i] = in ? (uint64_t)ga[abase[i] + (int64_t)k * AV.s1 + (int64_t)ys * AV.sy + (int64_t)xs * AV.sx] : 0;
        bv[u][i] = live ? (uint64_t)gk[kbase[i] + koff] : 0;
      }
      // advance (k, dy, dx) by the stride: each digit carries at most once
      dx += D.ddx;
      if (dx >= G.KW) {
        dx -= G.KW;
        ++dy;
      }
      dy += D.ddy;
      if (dy >= G.KH) {
        dy -= G.KH;
        ++k;
      }
      k += D.dk;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const uint32_t a0 = (uint32_t)(av[u][i] & kLo), a1 = (uint32_t)(av[u][i] >> 21);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const uint32_t b0 = (uint32_t)(bv[u][j] & kLo), b1 = (uint32_t)(bv[u][j] >> 21);
          s0[i * 2 + j] += (uint64_t)a0 * b0;
          s1[i * 2 + j] += (uint64_t)a0 * b1;
          s1[i * 2 + j] += (uint64_t)a1 * b0;
          s2[i * 2 + j] += (uint64_t)a1 * b1;
        }
      }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      s0[o] += __shfl_xor(s0[o], d);
      s1[o] += __shfl_xor(s1[o], d);
      s2[o] += __shfl_xor(s2[o], d);
    }
  // lane o < 4 takes output o = (row0 + o / 2, col0 + o % 2)
  uint64_t x0 = s0[0], x1 = s1[0], x2 = s2[0];
#pragma unroll
  for (int o = 1; o < 4; ++o)
    if (lane == o) {
      x0 = s0[o];
      x1 = s1[o];
      x2 = s2[o];
    }
  if constexpr (NWB == 4) {
    if (lane < 4) {
      red[wv][lane][0] = x0;
      red[wv][lane][1] = x1;
      red[wv][lane][2] = x2;
    }
    __syncthreads();
    if (wv != 0) return;
    if (lane < 4) {
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        x0 += red[w][lane][0];
        x1 += red[w][lane][1];
        x2 += red[w][lane][2];
      }
    }
  }
  if (lane >= 4) return;
  const int row = row0 + (lane >> 1), col = col0 + (lane & 1);
  if (row >= P || col >= R) return;
  const int m = WIN ? row / ohw : row, rem = row - m * ohw, y = WIN ? rem / G.OW : 0, x = rem - y * G.OW;
  // x0 + x1 2^21 + x2 2^42 as a 128-bit value, then mod t
  const uint64_t t1 = x1 << 21, t2 = x2 << 42;
  uint64_t lo = x0 + t1;
  uint64_t hi = (lo < t1 ? 1 : 0) + (x1 >> 43) + (x2 >> 22);
  lo += t2;
  hi += lo < t2 ? 1 : 0;
  gview(out)[(int64_t)m * OV.s0 + (int64_t)col * OV.s1 + (int64_t)y * OV.sy + (int64_t)x * OV.sx] =
      (int64_t)add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t), reduce64(lo, C.one_sh_t, C.t),
                       C.t);
}

// Z_t linear combination out = base + sum_i c_i x_i (mod t): the masked
// operands and share combinations of the preprocessed products (Pencil+,
// online phase).  Operands and coefficients are below t < 2^48, so each
// product fits 96 bits and 64 of them plus base fit 128.  The sum is a pure
// stream of loads, so a block holds 64 consecutive elements and kCombWaves
// waves: wave w takes the terms w, w + kCombWaves, ..., issues up to kCombUnroll
// of their loads before the first multiply, and the waves' 128-bit partial
// sums meet in LDS, where the first wave adds base and reduces mod t.
constexpr int kCombWaves = 8, kCombUnroll = 8;

__global__ void __launch_bounds__(64 * kCombWaves) k_zt_combine(ZtTerms T, const int64_t* base, int64_t* out,
                                                               int64_t count, Consts C) {
  __shared__ uint64_t part_lo[kCombWaves][64], part_hi[kCombWaves][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t g = (int64_t)blockIdx.x * 64 + lane;
  const bool live = g < count;
  uint64_t hi = 0, lo = 0;
  if (live) {
    for (int i0 = w; i0 < T.n; i0 += kCombWaves * kCombUnroll) {
      uint64_t x[kCombUnroll];
#pragma unroll
      for (int u = 0; u < kCombUnroll; ++u) {
        const int i = i0 + u * kCombWaves;
        x[u] = i < T.n ? (uint64_t)gview(T.x[i])[g] : 0;
      }
#pragma unroll
      for (int u = 0; u < kCombUnroll; ++u) {
        const int i = i0 + u * kCombWaves;
        if (i < T.n) {
          uint64_t ph, pl;
          mul_wide(x[u], T.c[i], ph, pl);
          lo += pl;
          hi += ph + (lo < pl ? 1 : 0);
        }
      }
    }
  }
  part_lo[w][lane] = lo;
  part_hi[w][lane] = hi;
  __syncthreads();
  if (w != 0 || !live) return;
  lo = base ? (uint64_t)gview(base)[g] : 0;
  hi = 0;
#pragma unroll
  for (int k = 0; k < kCombWaves; ++k) {
    const uint64_t pl = part_lo[k][lane];
    lo += pl;
    hi += part_hi[k][lane] + (lo < pl ? 1 : 0);
  }
  const uint64_t v = add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t),
                             reduce64(lo, C.one_sh_t, C.t), C.t);
  gview(out)[g] = (int64_t)v;
}

// ------------------------------------------ bias gradient and DP noise

// Bias gradient share (Sec. III.B.2): the sum of a dY share over the batch
// and, for a convolution, over the output positions, mod t.  dy is
// [batch][channels][spatial].  The host admits at most 2^(64 - bitlen(t))
// entries per channel, so a 64-bit total is exact until the final reduction.
__global__ void __launch_bounds__(256) k_bias_grad_cols(const int64_t* __restrict__ dy, int64_t* __restrict__ db,
                                                        int batch, int channels, Consts C) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= channels) return;
  const PENCIL_GLOBAL int64_t* p = gview(dy) + o;
  uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int b = 0;
  for (; b + 4 <= batch; b += 4) {
    a0 += (uint64_t)p[(int64_t)b * channels];
    a1 += (uint64_t)p[(int64_t)(b + 1) * channels];
    a2 += (uint64_t)p[(int64_t)(b + 2) * channels];
    a3 += (uint64_t)p[(int64_t)(b + 3) * channels];
  }
  for (; b < batch; ++b) a0 += (uint64_t)p[(int64_t)b * channels];
  gview(db)[o] = (int64_t)reduce64(a0 + a1 + a2 + a3, C.one_sh_t, C.t);
}

__global__ void __launch_bounds__(256) k_bias_grad_chan(const int64_t* __restrict__ dy, int64_t* __restrict__ db,
                                                        int batch, int channels, int spatial, Consts C) {
  __shared__ uint64_t part[256];
  const int o = blockIdx.x;
  const uint32_t total = (uint32_t)batch * (uint32_t)spatial;
  const PENCIL_GLOBAL int64_t* base = gview(dy) + (int64_t)o * spatial;
  const int64_t bstride = (int64_t)channels * spatial;
  uint64_t acc = 0;
  for (uint32_t i = threadIdx.x; i < total; i += 256) {
    const uint32_t b = i / (uint32_t)spatial, x = i - b * (uint32_t)spatial;
    acc += (uint64_t)base[(int64_t)b * bstride + x];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) gview(db)[o] = (int64_t)reduce64(part[0], C.one_sh_t, C.t);
}

// Gaussian perturbation the data owner adds to its weight-gradient and
// bias-gradient shares (Sec. III.B.2, DPSGD).  Box-Muller from Philox words,
// every step one IEEE double operation in a fixed order (contraction off), so
// the draws do not depend on the compiler's scheduling:
//   ln u, u = k 2^-53: u = m 2^e with m in [1/sqrt 2, sqrt 2), s = (m-1)/(m+1),
//     ln m = 2 s sum_{j<12} s^2j / (2j+1) (atanh series), ln u = e ln 2 + ln m;
//   cos, sin of 2 pi b 2^-53: quadrant q = round(b / 2^51), theta = (b - q 2^51)
//     2^-53 2 pi in [-pi/4, pi/4], Taylor series through theta^23, rotated by q.
struct DpCoeffs {
  double lg[12], cc[12], cs[12];
};

constexpr DpCoeffs make_dp_coeffs() {
  DpCoeffs c{};
  for (int j = 0; j < 12; ++j) c.lg[j] = 1.0 / (double)(2 * j + 1);
  c.cc[0] = 1.0;
  c.cs[0] = 1.0;
  for (int j = 1; j < 12; ++j) {
    c.cc[j] = c.cc[j - 1] / -(double)((2 * j - 1) * (2 * j));
    c.cs[j] = c.cs[j - 1] / -(double)((2 * j) * (2 * j + 1));
  }
  return c;
}

__device__ __forceinline__ double dp_pow2(int e) {  // 2^e for -1022 <= e <= 1023
  return __longlong_as_double((long long)((uint64_t)(1023 + e) << 52));
}

__device__ double dp_log_u(uint64_t k) {  // ln(k 2^-53), 1 <= k <= 2^53
#pragma clang fp contract(off)
  constexpr DpCoeffs K = make_dp_coeffs();
  constexpr double kSqrtHalf = 0.7071067811865476, kLn2 = 0.6931471805599453;
  const int bl = 64 - __clzll((long long)k);
  double m = (double)k * dp_pow2(-bl);
  int e = bl - 53;
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = K.lg[11];
#pragma unroll
  for (int j = 10; j >= 0; --j) p = p * s2 + K.lg[j];
  const double lnm = (s * p) * 2.0;
  return (double)e * kLn2 + lnm;
}

__device__ void dp_cos_sin_turns(uint64_t b, double& co, double& si) {  // of 2 pi b 2^-53, b < 2^53
#pragma clang fp contract(off)
  constexpr DpCoeffs K = make_dp_coeffs();
  constexpr double kTwoPi = 6.283185307179586;
  const int64_t bb = (int64_t)b;
  const int64_t q = (bb + (1ll << 50)) >> 51;
  const int64_t d = bb - (q << 51);
  const double theta = ((double)d * dp_pow2(-53)) * kTwoPi;
  const double t2 = theta * theta;
  double pc = K.cc[11], ps = K.cs[11];
#pragma unroll
  for (int j = 10; j >= 0; --j) {
    pc = pc * t2 + K.cc[j];
    ps = ps * t2 + K.cs[j];
  }
  const double c = pc, s = theta * ps;
  switch (q & 3) {
    case 0: co = c; si = s; break;
    case 1: co = -s; si = c; break;
    case 2: co = -c; si = -s; break;
    default: co = s; si = -c; break;
  }
}

__device__ __forceinline__ int64_t dp_add(int64_t x, double z, double sd, uint64_t t) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)floor(z * sd);
  int64_t em = e % (int64_t)t;
  if (em < 0) em += (int64_t)t;
  return (int64_t)add_mod((uint64_t)x, (uint64_t)em, t);
}

// One thread per Philox block: entries 4j .. 4j+3 from words (w0, w1), (w2, w3).
__global__ void __launch_bounds__(256) k_dp_noise(int64_t* __restrict__ x, int64_t count, double sd, uint64_t nonce,
                                                  uint64_t obj, Consts C) {
#pragma clang fp contract(off)
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = 4 * j;
  if (i0 >= count) return;
  const U64x4 w = philox((uint64_t)j, obj, P_DP, 0, C.seed, nonce);
  double z[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double r = sqrt(dp_log_u((w.v[2 * h] >> 11) + 1) * -2.0);
    double co, si;
    dp_cos_sin_turns(w.v[2 * h + 1] >> 11, co, si);
    z[2 * h] = r * co;
    z[2 * h + 1] = r * si;
  }
  PENCIL_GLOBAL int64_t* px = gview(x) + i0;
#pragma unroll
  for (int h = 0; h < 4; ++h)
    if (i0 + h < count) px[h] = dp_add(px[h], z[h], sd, C.t);
}

// ------------------------------------------------- stride-s relayouts

// A stride-s correlation equals a stride-1 correlation over the space-to-depth
// image: channel c' = c sy sx + a sx + e holds Xpad[., c, sy y + a, sx x + e]
// and the kernel W[., c, sy i + a, sx j + e] (zero past the kernel's edge).
// Each mode gathers one output entry per thread; padding and taps that fall
// outside either tensor read as zero.
__global__ void __launch_bounds__(256) k_stride_relayout(Relayout R, const int64_t* __restrict__ in,
                                                         int64_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= R.total) return;
  const int ss = R.sy * R.sx;
  int64_t v = 0;
  if (R.mode == 0 || R.mode == 1) {  // out [n][c * ss][Y][X] from in [n][c][.][.]
    const int Y = R.mode == 0 ? R.h2 : R.kh2, X = R.mode == 0 ? R.w2 : R.kw2;
    const int x2 = (int)(g % X);
    int64_t r = g / X;
    const int y2 = (int)(r % Y);
    r /= Y;
    const int c2 = (int)(r % ((int64_t)R.ci * ss));
    const int64_t n = r / ((int64_t)R.ci * ss);
    const int c = c2 / ss, a = (c2 / R.sx) % R.sy, e = c2 % R.sx;
    if (R.mode == 0) {
      const int yy = R.sy * y2 + a - R.ph, xx = R.sx * x2 + e - R.pw;
      if (yy >= 0 && yy < R.h && xx >= 0 && xx < R.w)
        v = gview(in)[((n * R.ci + c) * R.h + yy) * R.w + xx];
    } else {
      const int i = R.sy * y2 + a, j = R.sx * x2 + e;
      if (i < R.kh && j < R.kw) v = gview(in)[((n * R.ci + c) * R.kh + i) * R.kw + j];
    }
  } else {  // out [n][c][Y][X] from in [n][c * ss][.][.]
    const int Y = R.mode == 2 ? R.h : R.kh, X = R.mode == 2 ? R.w : R.kw;
    const int x = (int)(g % X);
    int64_t r = g / X;
    const int y = (int)(r % Y);
    r /= Y;
    const int c = (int)(r % R.ci);
    const int64_t n = r / R.ci;
    const int yy = R.mode == 2 ? y + R.ph : y, xx = R.mode == 2 ? x + R.pw : x;
    const int y2 = yy / R.sy, x2 = xx / R.sx, c2 = c * ss + (yy % R.sy) * R.sx + xx % R.sx;
    const int Y2 = R.mode == 2 ? R.h2 : R.kh2, X2 = R.mode == 2 ? R.w2 : R.kw2;
    if (y2 < Y2 && x2 < X2) v = gview(in)[((n * ((int64_t)R.ci * ss) + c2) * Y2 + y2) * X2 + x2];
  }
  gview(out)[g] = v;
}

// Every flood-and-mask of one step, for one flood width.
template <int W>
__global__ void __launch_bounds__(256) k_step_flood(const StepSeg* __restrict__ segs, int nseg,
                                                    const Consts* __restrict__ consts,
                                                    const uint64_t* __restrict__ nonce) {
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const int64_t g = ((int64_t)blockIdx.x - S.block_begin) * blockDim.x + threadIdx.x;
  do_flood<W>(S.dst, S.count, S.share, S.bias, S.G, S.V2, *nonce + S.nonce_off, S.obj_base, consts[S.ctx], g);
}

__global__ void k_set_u64(uint64_t* p, uint64_t v, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = add ? p[0] + v : v;
}

hipError_t launch_flood_mask(uint64_t* ct, int64_t n_out, int64_t* share0, const int64_t* bias, const Geo& G,
                             const View& outV, uint64_t nonce, uint64_t obj_base, const Consts& C, hipStream_t s) {
  if (n_out <= 0) return hipSuccess;
  const int64_t threads = n_out * (C.n / 4);
  const dim3 grid((unsigned)((threads + 255) / 256));
  switch (C.flood_words) {
    case 1: hipLaunchKernelGGL(k_flood_mask<1>, grid, dim3(256), 0, s, ct, n_out, share0, bias, G, outV, nonce, obj_base, C); break;
    case 2: hipLaunchKernelGGL(k_flood_mask<2>, grid, dim3(256), 0, s, ct, n_out, share0, bias, G, outV, nonce, obj_base, C); break;
    case 3: hipLaunchKernelGGL(k_flood_mask<3>, grid, dim3(256), 0, s, ct, n_out, share0, bias, G, outV, nonce, obj_base, C); break;
    case 4: hipLaunchKernelGGL(k_flood_mask<4>, grid, dim3(256), 0, s, ct, n_out, share0, bias, G, outV, nonce, obj_base, C); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zt_combine(const ZtTerms& T, const int64_t* base, int64_t* out, int64_t count, const Consts& C,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zt_combine, dim3((unsigned)((count + 63) / 64)), dim3(64 * kCombWaves), 0, s, T, base, out,
                     count, C);
  return hipGetLastError();
}

hipError_t launch_bias_grad(const int64_t* dy, int64_t* db, int batch, int channels, int spatial, const Consts& C,
                            hipStream_t s) {
  if (channels <= 0) return hipSuccess;
  if (spatial == 1)
    hipLaunchKernelGGL(k_bias_grad_cols, dim3((unsigned)((channels + 255) / 256)), dim3(256), 0, s, dy, db, batch,
                       channels, C);
  else
    hipLaunchKernelGGL(k_bias_grad_chan, dim3((unsigned)channels), dim3(256), 0, s, dy, db, batch, channels, spatial,
                       C);
  return hipGetLastError();
}

hipError_t launch_dp_noise(int64_t* x, int64_t count, double sd, uint64_t nonce, uint64_t obj, const Consts& C,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t threads = (count + 3) / 4;
  hipLaunchKernelGGL(k_dp_noise, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, x, count, sd, nonce, obj,
                     C);
  return hipGetLastError();
}

hipError_t launch_stride_relayout(const Relayout& R, const int64_t* in, int64_t* out, hipStream_t s) {
  if (R.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stride_relayout, dim3((unsigned)((R.total + 255) / 256)), dim3(256), 0, s, R, in, out);
  return hipGetLastError();
}

constexpr int64_t kDotMinK = 256, kDotWideK = 8192, kDotMaxTiles = 64, kMfmaMinTiles = 256, kMfmaMinWaves = 512;
constexpr int kDotMaxSkinny = 4;

hipError_t launch_zt_corr(const int64_t* a, const int64_t* k, int64_t* out, const Geo& G, const View& AV,
                          const View& KV, const View& OV, const Consts& C, hipStream_t s) {
  const int64_t total = (int64_t)G.M * G.R * G.OH * G.OW;
  if (total <= 0) return hipSuccess;
  const int64_t rows = (int64_t)G.M * G.OH * G.OW, ctot = (int64_t)G.K * G.KH * G.KW;
  // Tiled kernel: 2 x 2 outputs per lane when that still gives >= 512
  // workgroups, else 1; about 16 contraction steps per wave, at most 16 waves.
  // Operands split at bit 21 (high part h = bitlen(t) - 21 bits): a partial
  // sum takes terms below 2^42, 2^(22 + h) and 2^(2h), so a wave may sum
  // 2^(64 - max) of them (2^22 for t < 2^42).
  const int tb = 64 - __builtin_clzll(C.t), hb = tb > 21 ? tb - 21 : 0;
  const int mb = std::max(42, std::max(22 + hb, 2 * hb));
  const int64_t per_wave_max = mb >= 63 ? 1 : (int64_t)1 << (64 - mb);
  const int64_t tiles = ((rows + 15) / 16) * ((G.R + 15) / 16);
  // Long contractions whose outputs fill few 16 x 16 tiles, or only a few
  // columns of each (at most kDotMaxSkinny, where the other kernels' tiles
  // would compute mostly padding): 2 x 2 output blocks, the lanes of one wave
  // (or, from kDotWideK indices, of four waves) splitting the contraction,
  // whose whole length one partial sum then holds.
  if (ctot >= kDotMinK && (tiles < kDotMaxTiles || G.R <= kDotMaxSkinny) && ctot <= per_wave_max) {
    const int64_t blocks = (int64_t)((rows + 1) / 2) * ((G.R + 1) / 2);
    const int nwb = ctot >= kDotWideK ? 4 : 1;
    const int kk = G.KH * G.KW, st = 64 * nwb;
    const DotStep D{st / kk, (st % kk) / G.KW, (st % kk) % G.KW, 0};
    const int64_t grid = nwb == 4 ? blocks : (blocks + 3) / 4;
    const bool win = !(kk == 1 && G.OH == 1 && G.OW == 1 && AV.H == 1 && AV.W == 1 && AV.pad == 0 && AV.pady == 0);
    if (grid < (1ll << 31)) {
      const dim3 g((unsigned)grid), b(256);
      if (nwb == 4 && win)
        hipLaunchKernelGGL((k_zt_dot<4, true>), g, b, 0, s, a, k, out, G, AV, KV, OV, C, D);
      else if (nwb == 4)
        hipLaunchKernelGGL((k_zt_dot<4, false>), g, b, 0, s, a, k, out, G, AV, KV, OV, C, D);
      else if (win)
        hipLaunchKernelGGL((k_zt_dot<1, true>), g, b, 0, s, a, k, out, G, AV, KV, OV, C, D);
      else
        hipLaunchKernelGGL((k_zt_dot<1, false>), g, b, 0, s, a, k, out, G, AV, KV, OV, C, D);
      return hipGetLastError();
    }
  }
  // Matrix-core kernel, one 16 x 16 output tile per workgroup: four
  // contraction indices per step, about eight steps per wave, at most 16
  // waves.  A wave may run 2^53 / (4 * 2^termb) steps, termb bounding a
  // diagonal's per-index term: with two 21-bit digits (t < 2^42; top digit
  // below 2^(bitlen(t) - 22)) 2^42; with three 14-bit digits 2^30 (t < 2^43;
  // 2^(2 bitlen(t) - 58) above).  Taken when its grid has at least
  // kMfmaMinTiles tiles or kMfmaMinWaves waves; smaller grids measured faster
  // on the vector kernel, whose 8 x 8 tiles spread the work over more waves.
  {
    const int64_t steps = (ctot + 3) / 4;
    const int nwm = (int)std::min<int64_t>(kZtWaves, std::max<int64_t>(1, steps / 8));
    const int64_t per = (steps + nwm - 1) / nwm;
    const int64_t gx = (rows + 15) / 16, gy = ((int64_t)G.R + 15) / 16;
    const int d2b = tb > 29 ? tb - 29 : 0;  // bits of the top 14-bit-split digit
    const int termb3 = std::max(30, std::max(tb - 13, 2 * d2b));
    const int64_t max3 = termb3 >= 51 ? 0 : (int64_t)1 << (51 - termb3);
    const int64_t max2 = tb <= 42 ? (int64_t)1 << (51 - 42) : 0;
    if ((tiles >= kMfmaMinTiles || tiles * nwm >= kMfmaMinWaves) && gx < (1ll << 31) && gy < 65536) {
      const dim3 grid((unsigned)gx, (unsigned)gy), block(64 * nwm);
      if (per <= max2) {
        hipLaunchKernelGGL(k_zt_mfma<2>, grid, block, 0, s, a, k, out, G, AV, KV, OV, C);
        return hipGetLastError();
      }
      if (per <= max3) {
        hipLaunchKernelGGL(k_zt_mfma<3>, grid, block, 0, s, a, k, out, G, AV, KV, OV, C);
        return hipGetLastError();
      }
    }
  }
  const int ti = tiles >= 512 ? 2 : 1;
  const int64_t steps16 = ctot / 16;
  const int nw = steps16 < 1 ? 1 : steps16 > kZtWaves ? kZtWaves : (int)steps16;
  const int64_t gx = (rows + 8 * ti - 1) / (8 * ti), gy = ((int64_t)G.R + 8 * ti - 1) / (8 * ti);
  if ((ctot + nw - 1) / nw <= per_wave_max && gx < (1ll << 31) && gy < 65536) {
    const dim3 grid((unsigned)gx, (unsigned)gy);
    if (ti == 2)
      hipLaunchKernelGGL(k_zt_gemm<2>, grid, dim3(64 * nw), 0, s, a, k, out, G, AV, KV, OV, C);
    else
      hipLaunchKernelGGL(k_zt_gemm<1>, grid, dim3(64 * nw), 0, s, a, k, out, G, AV, KV, OV, C);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_zt_corr, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, k, out, G, AV, KV, OV, C);
  return hipGetLastError();
}

hipError_t launch_step_flood(int words, const StepPhase& P, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  switch (words) {
    case 1: hipLaunchKernelGGL(k_step_flood<1>, dim3((unsigned)blocks), dim3(256), 0, s, P.segs, P.nseg, P.consts, P.nonce); break;
    case 2: hipLaunchKernelGGL(k_step_flood<2>, dim3((unsigned)blocks), dim3(256), 0, s, P.segs, P.nseg, P.consts, P.nonce); break;
    case 3: hipLaunchKernelGGL(k_step_flood<3>, dim3((unsigned)blocks), dim3(256), 0, s, P.segs, P.nseg, P.consts, P.nonce); break;
    case 4: hipLaunchKernelGGL(k_step_flood<4>, dim3((unsigned)blocks), dim3(256), 0, s, P.segs, P.nseg, P.consts, P.nonce); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t* p, uint64_t v, int add, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, p, v, add);
  return hipGetLastError();
}

// ------------------------------------------------ fixed point and sharing
// Fixed-point values carried in float64 (integers, |x| < 2^53) to Z_t: round to
// nearest (ties to even), then reduce mod t.
__global__ void __launch_bounds__(256) k_zt_encode(const double* __restrict__ x, int64_t* __restrict__ out,
                                                   int64_t count, int64_t t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int64_t v = __double2ll_rn(gview(x)[i]) % t;
  gview(out)[i] = v < 0 ? v + t : v;
}

// Z_t to the centred representative in float64: v - t above (t - 1) / 2.
__global__ void __launch_bounds__(256) k_zt_decode(const int64_t* __restrict__ v, double* __restrict__ out,
                                                   int64_t count, int64_t t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t a = gview(v)[i];
  gview(out)[i] = (double)(a > (t - 1) / 2 ? a - t : a);
}

// Additive shares over Z_t: s0 uniform (entry i from stream words 2i, 2i+1 of
// (nonce, object, P_SHARE), a 128-bit integer reduced mod t), s1 = v - s0.
// Each thread draws one Philox block, two entries.
__global__ void __launch_bounds__(256) k_zt_share(const int64_t* __restrict__ v, int64_t* __restrict__ s0,
                                                  int64_t* __restrict__ s1, int64_t count, uint64_t nonce,
                                                  uint64_t obj, Consts C) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * b >= count) return;
  const U64x4 w = philox((uint64_t)b, obj, P_SHARE, 0, C.seed, nonce);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t i = 2 * b + h;
    if (i >= count) break;
    const uint64_t hi = reduce64(w.v[2 * h + 1], C.one_sh_t, C.t);
    uint64_t r = mul_shoup(hi, C.r64t, C.r64t_sh, C.t) + reduce64(w.v[2 * h], C.one_sh_t, C.t);
    if (r >= C.t) r -= C.t;
    const uint64_t x = (uint64_t)gview(v)[i];
    gview(s0)[i] = (int64_t)r;
    gview(s1)[i] = (int64_t)(x >= r ? x - r : x + C.t - r);
  }
}

hipError_t launch_zt_encode(const double* x, int64_t* out, int64_t count, const Consts& C, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zt_encode, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, x, out, count,
                     (int64_t)C.t);
  return hipGetLastError();
}

hipError_t launch_zt_decode(const int64_t* v, double* out, int64_t count, const Consts& C, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zt_decode, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, v, out, count,
                     (int64_t)C.t);
  return hipGetLastError();
}

hipError_t launch_zt_share(const int64_t* v, int64_t* s0, int64_t* s1, int64_t count, uint64_t nonce, uint64_t obj,
                           const Consts& C, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t pairs = (count + 1) / 2;
  hipLaunchKernelGGL(k_zt_share, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, v, s0, s1, count, nonce,
                     obj, C);
  return hipGetLastError();
}

// ------------------------------------------------ integer multiply probe
// Issue rate of one 32-bit multiply form (the integer roofline's peak): each
// thread runs 8 independent dependent chains of `iters` instructions.  Kind 0:
// v_mad_u64_u32 (acc = lo32(acc) * a + acc), 1: v_mul_lo_u32, 2: v_mul_hi_u32.
template <int KIND>
__global__ void __launch_bounds__(256) k_probe_mul(uint64_t* out, uint32_t seed, int iters) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[8];
  uint64_t x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (seed ^ (g * 8u + (uint32_t)i)) | 0x80000001u;
    x[i] = a[i] * 0x9E3779B9u + (uint64_t)i;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (KIND == 0) x[i] = (uint64_t)(uint32_t)x[i] * a[i] + x[i];
      if (KIND == 1) x[i] = (uint32_t)x[i] * a[i];
      if (KIND == 2) x[i] = __umulhi((uint32_t)x[i], a[i]);
    }
  }
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) sum ^= x[i];
  out[g] = sum;
}

hipError_t launch_probe_mul(int kind, uint64_t* out, int64_t threads, int iters, hipStream_t s) {
  const dim3 grid((unsigned)(threads / 256)), block(256);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_probe_mul<0>, grid, block, 0, s, out, 12345u, iters); break;
    case 1: hipLaunchKernelGGL(k_probe_mul<1>, grid, block, 0, s, out, 12345u, iters); break;
    case 2: hipLaunchKernelGGL(k_probe_mul<2>, grid, block, 0, s, out, 12345u, iters); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------ allocation-free scratch
// The scratch memory of the allocation-free entry points: a file-scope device
// array, so each GPU the library runs on holds its own copy from the moment
// the code object is loaded until the process ends.  In host code the array's
// name is a host-side stand-in, not a device address: only the address
// hipGetSymbolAddress returns (per device, with that device current) is ever
// passed to a kernel.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t configure_lds_limits() {
  hipError_t e[4] = {configure_lds_ntt(), configure_lds_mac(), configure_lds_do(), configure_lds_step()};
  for (hipError_t x : e)
    if (x != hipSuccess) return x;
  return hipSuccess;
}

}  // namespace pencil
