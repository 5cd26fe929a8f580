// Batched step: every forward and inverse NTT of a step's products, one
// launch per ring degree, over a device-side segment table.
#include "ntt_core.h"

namespace pencil {

// Every NTT of one phase, for one ring degree: the forward transforms of the
// inputs (k_step_ntt: ciphertexts, plaintexts, re-randomisation masks) or the
// inverse transforms of the outputs (k_step_intt).
template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE)
    k_step_ntt(const StepSeg* __restrict__ segs, int nseg, const Consts* __restrict__ consts,
               const Tables* __restrict__ tabs, const uint64_t* __restrict__ nonce) {
  extern __shared__ uint64_t lds[];
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const Consts& C = consts[S.ctx];
  const Tables& T = tabs[S.ctx];
  const int64_t p = (int64_t)blockIdx.x - S.block_begin;
  switch (S.kind) {
    case SEG_CT: do_ntt_ct<LOGN, LOGE>(lds, S.src, S.dst, S.tensor, S.G, S.V, C, T, p); break;
    case SEG_PT: do_ntt_pt<LOGN, LOGE>(lds, S.tensor, S.dst, S.side, S.G, S.V, C, T, p); break;
    case SEG_TERN: do_ntt_ternary<LOGN, LOGE>(lds, S.dst, *nonce + S.nonce_off, S.obj_base, S.purpose, 1, C, T, p); break;
    default: break;
  }
}

template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE)
    k_step_intt(const StepSeg* __restrict__ segs, int nseg, const Consts* __restrict__ consts,
                const Tables* __restrict__ tabs) {
  extern __shared__ uint64_t lds[];
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const int64_t p = (int64_t)blockIdx.x - S.block_begin;
  do_ntt_plain<LOGN, LOGE>(lds, S.dst, 1, consts[S.ctx], tabs[S.ctx], p);
}

hipError_t launch_step_ntt(int log2n, int loge, bool inverse, const StepPhase& P, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  Consts C{};  // only log2n, n and ntt_loge are read by the dispatch
  C.log2n = log2n;
  C.n = 1 << log2n;
  C.ntt_loge = loge;
  const dim3 grid((unsigned)blocks);
  if (inverse)
    NTT_DISPATCH(k_step_intt, grid, C, s, P.segs, P.nseg, P.consts, P.tabs);
  else
    NTT_DISPATCH(k_step_ntt, grid, C, s, P.segs, P.nseg, P.consts, P.tabs, P.nonce);
  return hipGetLastError();
}

hipError_t configure_lds_step() {
  const int max_lds = 160 * 1024;
  hipError_t e = hipSuccess;
#define PENCIL_RAISE(LN, LE)                                                                            \
  for (const void* f : {(const void*)k_step_ntt<LN, LE>, (const void*)k_step_intt<LN, LE>}) {           \
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);         \
    if (r != hipSuccess) e = r;                                                                          \
  }
  PENCIL_RAISE(13, 4)
  PENCIL_RAISE(13, 5)
  PENCIL_RAISE(14, 4)
  PENCIL_RAISE(14, 5)
#undef PENCIL_RAISE
  return e;
}

}  // namespace pencil
