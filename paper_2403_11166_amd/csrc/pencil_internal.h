// Internal types shared by the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pencil {

constexpr int kMaxLimbs = 4;
constexpr int kMaxWords = 5;  // multiword integers up to 320 bits (q < 2^244)

// Per-RNS-limb constants.  "_sh" fields are Shoup companions floor(w * 2^64 / q).
struct LimbConst {
  uint64_t q;
  uint64_t r64, r64_sh;          // 2^64 mod q
  uint64_t r128, r192;           // 2^128 mod q, 2^192 mod q
  uint64_t one_sh;               // floor(2^64 / q)
  uint64_t ninv, ninv_sh;        // N^-1 mod q
  uint64_t delta, delta_sh;      // floor(q / t) mod q_l
  uint64_t t_sh;                 // floor(t * 2^64 / q_l), t < q_l
  uint64_t qhat_inv, qhat_inv_sh;// ((q / q_l)^-1) mod q_l
  uint64_t flood_off;            // 2^fb mod q_l
  uint64_t mu_lo, mu_hi;         // floor(2^128 / q_l), for 128-bit Barrett reduction
};

// Everything a kernel needs about the parameter set; passed by value.
struct Consts {
  int32_t log2n, n, L, flood_words;
  uint32_t flood_bits, mac_chunk, qwords;
  int32_t ntt_loge;              // log2 of the residues each NTT thread keeps (4 or 5)
  uint32_t mac_fold, mac_fold4;  // MAC steps per fold of the 64-bit partial sums (three, four sums)
  uint64_t t, t_half;            // t and (t - 1) / 2
  uint64_t rho, rho_sh;          // q mod t, floor(rho * 2^64 / t)
  uint64_t r64t, r64t_sh;        // 2^64 mod t and floor(r64t * 2^64 / t)
  uint64_t one_sh_t;             // floor(2^64 / t)
  uint64_t top_mask;             // mask of the flood's top word
  uint64_t seed;
  LimbConst limb[kMaxLimbs];
  uint64_t qhat[kMaxLimbs][kMaxWords];  // q / q_l, little-endian words
  uint64_t thr[kMaxLimbs][kMaxWords];   // (2j + 1) * q, j = 0..L-1
};

// A twiddle and its Shoup companion, stored together for one 16-byte load.
struct alignas(16) TW {
  uint64_t w, ws;
};

// NTT tables, each [L][N]: psi^rev(k) (forward) and psi^-rev(k) (inverse).
struct Tables {
  const TW* fw;
  const TW* iw;
};

// Partition of one packed correlation into N-slot tiles.
struct Geo {
  int32_t M, R, K, HA, WA, KH, KW, OH, OW;      // virtual operand dims
  int32_t mt, rt, kt, oh, ow, kh, kw, ha, wa;   // tile dims (ha = oh + kh - 1)
  int32_t nM, nR, nK, nOY, nOX, nKY, nKX;       // tile counts
  int32_t S;                                    // kt * ha * wa
  int32_t RS;                                   // rt * S: stride of m inside a tile
  int32_t O;                                    // reverse-encoding offset
  int32_t pad1;
  // Reciprocals ceil(2^32 / d) of the in-tile divisors d = RS, ha*wa, wa and S,
  // and of kw, kh*kw, kt*kh*kw for enumerating a K tile's entries (0 for
  // d = 1): floor(n / d) = umulhi(n, m) for n, d < 2^16.
  uint32_t dv_rs, dv_hw, dv_wa, dv_s;
  uint32_t dv_kw, dv_khw, dv_kthw, pad2;
};

// Maps virtual coordinates (i0, i1, y, x) of an operand to an element offset of
// the caller's tensor.  A side: y, x are shifted by -pad and bounded by H, W.
// K side: flip mirrors the kernel window.  Output: plain strides.
struct View {
  int64_t s0, s1, sy, sx;
  int32_t pad, H, W, flip;   // pad: zero columns before the tensor (and rows, see pady)
  int32_t KH, KW, pady, pad3;
};

// Philox stream purposes.
enum Purpose : uint32_t {
  P_SK = 1, P_PK_A = 2, P_PK_E = 3,
  P_ENC_U = 16, P_ENC_E0 = 17, P_ENC_E1 = 18,
  P_RR_U = 32, P_RR_E0 = 33, P_RR_E1 = 34, P_FLOOD = 35, P_MASK = 36,
  P_DP = 48, P_SHARE = 49,
};
constexpr uint64_t kKeygenNonce = ~0ull;

inline uint64_t enc_object(int operand, uint64_t i) { return ((uint64_t)(operand + 1) << 48) | i; }
inline uint64_t out_object(int op, uint64_t i) { return ((uint64_t)(op + 5) << 48) | i; }

// One term of a product: which side holds the ciphertext and where both operands live
// (NTT domain, split form).  ct: [n][2][L][N] (component 0 addresses); pt: [n][L][N].
// A ciphertext's component 1 sits c1 elements after its component 0: L*N in the
// caller's buffer, or elsewhere when component 0 is a staged copy with the
// model owner's share added.
struct MacTerm {
  const uint64_t* a;   // A-side tiles
  const uint64_t* k;   // K-side tiles
  int64_t c1;          // component-1 offset on the ciphertext side (elements)
  int32_t a_is_ct;     // 1: A side is a ciphertext, K side a plaintext; 0: the reverse
  int32_t pad;
};

struct MacArgs {
  MacTerm term[2];
  int32_t n_terms;
  int32_t m_rows;      // nM * nOY * nOX
  int32_t variant;     // multiply-accumulate schedule (0..kMacVariants-1), see mac_rows
  int32_t pad;
  const uint64_t* pk;  // [2][L][N], NTT domain, split form
  const uint64_t* u;   // [n_out][L][N], NTT domain
  uint64_t* out;       // [n_out][2][L][N]
};

// A batched step runs every product of several layers as a few phase launches.
// Each phase launch covers a list of segments; a segment is a contiguous range
// of blocks that share their arguments (one operand's NTTs, one op's MAC, ...).
enum SegKind : int32_t { SEG_CT = 0, SEG_PT = 1, SEG_TERN = 2, SEG_INTT = 3, SEG_MAC = 4, SEG_FLOOD = 5 };

struct StepSeg {
  int64_t block_begin;       // first block of the segment in its phase grid
  int32_t kind, ctx, side, purpose;
  int64_t count;             // flood: number of output ciphertexts
  int64_t slot_blocks;       // mac: 64-slot groups (work items = slot_blocks x chunks)
  uint64_t nonce_off, obj_base;
  const uint64_t* src;
  uint64_t* dst;
  const int64_t* tensor;
  const int64_t* bias;
  int64_t* share;
  Geo G;
  View V, V2;
  MacArgs mac;
};

struct StepPhase {
  const StepSeg* segs;
  int32_t nseg, pad;
  const Consts* consts;      // per context of the step
  const Tables* tabs;
  const uint64_t* nonce;     // base nonce in device memory
};

// Output-chunk shape of each MAC variant and the number of chunks it needs.
// Variant v = 3 kind + shape.  Every wave accumulates a 2 x 2 block of
// (A row, K row) outputs.  Kind 0 stages operands in LDS, kind 1 loads them
// directly, both for the two ciphertext components; kind 2 loads directly for
// one component (the block's waves alternate components).  The shape picks the
// chunk (A rows x K rows) of the block's 8 waves: 4 x 8, 2 x 16, 8 x 4
// (kinds 0, 1) or 4 x 4, 2 x 8, 8 x 2 (kind 2).
constexpr int kMacVariants = 9;
__host__ __device__ inline int mac_rows(int variant) { return variant % 3 == 1 ? 2 : variant % 3 == 2 ? 8 : 4; }
__host__ __device__ inline int mac_cols(int variant) {
  const int c = variant % 3 == 1 ? 16 : variant % 3 == 2 ? 4 : 8;
  return variant >= 6 ? c / 2 : c;
}
__host__ __device__ inline int mac_chunks(int variant, int m_rows, int n_r) {
  return ((m_rows + mac_rows(variant) - 1) / mac_rows(variant)) * ((n_r + mac_cols(variant) - 1) / mac_cols(variant));
}

// ---------------------------------------------------------------- launchers
// (defined in kernels.hip; all enqueue on `stream` and return the launch status)
hipError_t launch_ntt_plain(uint64_t* data, int64_t polys, bool inverse, const Consts& C, const Tables& T,
                            hipStream_t s);
hipError_t launch_ntt_ct(const uint64_t* src, uint64_t* dst, int64_t n_ct, const int64_t* share, const Geo& G,
                         const View& V, const Consts& C, const Tables& T, hipStream_t s);
hipError_t launch_ntt_pt(const int64_t* tensor, uint64_t* dst, int64_t n_pt, int side, const Geo& G, const View& V,
                         const Consts& C, const Tables& T, hipStream_t s);
hipError_t launch_ntt_ternary(uint64_t* dst, int64_t count, uint64_t nonce, uint64_t obj_base, uint32_t purpose, int split,
                              const Consts& C, const Tables& T, hipStream_t s);
hipError_t launch_mac(const MacArgs& A, int64_t n_out, const Geo& G, const Consts& C, hipStream_t s);
hipError_t launch_flood_mask(uint64_t* ct, int64_t n_out, int64_t* share0, const int64_t* bias, const Geo& G,
                             const View& outV, uint64_t nonce, uint64_t obj_base, const Consts& C, hipStream_t s);
hipError_t launch_encrypt(const uint64_t* u_ntt, const int64_t* share, uint64_t* ct, int64_t n_ct, int side,
                          const Geo& G, const View& V, const uint64_t* pk_ntt, const uint64_t* pk_sh, uint64_t nonce,
                          uint64_t obj_base, const Consts& C, const Tables& T, hipStream_t s);
hipError_t launch_phase(const uint64_t* ct, uint64_t* x, int64_t n_ct, const uint64_t* s_ntt, const uint64_t* s_sh,
                        const Consts& C, const Tables& T, hipStream_t s);
hipError_t launch_decode(const uint64_t* x, int64_t* share, int64_t n_out, const Geo& G, const View& outV,
                         const Consts& C, uint32_t* noise, hipStream_t s);
// Up to kZtTerms terms of a Z_t linear combination, by value (kernel argument).
constexpr int kZtTerms = 64;
struct ZtTerms {
  const int64_t* x[kZtTerms];
  uint64_t c[kZtTerms];
  int32_t n, pad;
};
hipError_t launch_zt_combine(const ZtTerms& T, const int64_t* base, int64_t* out, int64_t count, const Consts& C,
                             hipStream_t s);
hipError_t launch_bias_grad(const int64_t* dy, int64_t* db, int batch, int channels, int spatial, const Consts& C,
                            hipStream_t s);
hipError_t launch_dp_noise(int64_t* x, int64_t count, double sd, uint64_t nonce, uint64_t obj, const Consts& C,
                           hipStream_t s);

// Space-to-depth relayout between a stride-s layer and its stride-1
// equivalent.  mode 0: X -> X', 1: W -> W', 2: dX' -> dX, 3: dW' -> dW.
struct Relayout {
  int32_t mode, batch, ci, co;
  int32_t h, w, kh, kw;   // the strided layer: input, kernel
  int32_t sy, sx, ph, pw; // stride and padding per axis (sy = 1 for conv1d)
  int32_t h2, w2, kh2, kw2;  // the equivalent layer: input, kernel
  int64_t total;          // entries of the output tensor
};
hipError_t launch_stride_relayout(const Relayout& R, const int64_t* in, int64_t* out, hipStream_t s);
hipError_t launch_zt_corr(const int64_t* a, const int64_t* k, int64_t* out, const Geo& G, const View& AV,
                          const View& KV, const View& OV, const Consts& C, hipStream_t s);
hipError_t launch_step_ntt(int log2n, int loge, bool inverse, const StepPhase& P, int64_t blocks, hipStream_t s);
hipError_t launch_step_mac(const StepPhase& P, int64_t blocks, int kind, hipStream_t s);
hipError_t launch_step_flood(int words, const StepPhase& P, int64_t blocks, hipStream_t s);
hipError_t launch_set_u64(uint64_t* p, uint64_t v, int add, hipStream_t s);
hipError_t launch_keygen(uint64_t* s_ntt, int64_t* s_coeff, uint64_t* pk_coeff, uint64_t* pk_ntt,
                         const Consts& C, const Tables& T, hipStream_t s);

// Fixed point (float64 integers <-> Z_t, centred) and additive sharing.
hipError_t launch_zt_encode(const double* x, int64_t* out, int64_t count, const Consts& C, hipStream_t s);
hipError_t launch_zt_decode(const int64_t* v, double* out, int64_t count, const Consts& C, hipStream_t s);
hipError_t launch_zt_share(const int64_t* v, int64_t* s0, int64_t* s1, int64_t count, uint64_t nonce, uint64_t obj,
                           const Consts& C, hipStream_t s);

// Multiply probe: `threads` (a multiple of 256) threads, 8 chains of `iters`
// instructions of kind 0 (v_mad_u64_u32), 1 (v_mul_lo_u32) or 2
// (v_mul_hi_u32) each; out receives one word per thread.
hipError_t launch_probe_mul(int kind, uint64_t* out, int64_t threads, int iters, hipStream_t s);

// Scratch array of the allocation-free entry points (one per GPU, in the
// library's code object): kScratchBytes, 256-byte aligned.  scratch_address
// returns its device address on `device`, which must be the current device;
// the address is looked up once per device and kept.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_address(int device, void** out);

// Kernels that stage more than 64 KiB of LDS opt in once per process; one
// function per translation unit, all called by configure_lds_limits().
hipError_t configure_lds_ntt();
hipError_t configure_lds_mac();
hipError_t configure_lds_do();
hipError_t configure_lds_step();
hipError_t configure_lds_limits();

}  // namespace pencil
