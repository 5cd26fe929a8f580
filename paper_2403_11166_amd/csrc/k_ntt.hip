// Per-call NTT kernels: plain transforms and the forward-transform front ends
// of one product.
#include "ntt_core.h"

namespace pencil {

template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE) k_ntt_plain(uint64_t* data, int inverse, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  do_ntt_plain<LOGN, LOGE>(lds, data, inverse, C, T, blockIdx.x);
}

template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE) k_ntt_ct(const uint64_t* src, uint64_t* dst, const int64_t* share, Geo G,
                                                 View V, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  do_ntt_ct<LOGN, LOGE>(lds, src, dst, share, G, V, C, T, blockIdx.x);
}

template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE) k_ntt_pt(const int64_t* tensor, uint64_t* dst, int side, Geo G, View V,
                                                 Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  do_ntt_pt<LOGN, LOGE>(lds, tensor, dst, side, G, V, C, T, blockIdx.x);
}

template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE) k_ntt_ternary(uint64_t* dst, uint64_t nonce, uint64_t obj_base,
                                                      uint32_t purpose, int split, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  do_ntt_ternary<LOGN, LOGE>(lds, dst, nonce, obj_base, purpose, split, C, T, blockIdx.x);
}

hipError_t launch_ntt_plain(uint64_t* data, int64_t polys, bool inverse, const Consts& C, const Tables& T,
                            hipStream_t s) {
  if (polys <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_plain, dim3((unsigned)(polys * C.L)), C, s, data, inverse ? 1 : 0, C, T);
  return hipGetLastError();
}

hipError_t launch_ntt_ct(const uint64_t* src, uint64_t* dst, int64_t n_ct, const int64_t* share, const Geo& G,
                         const View& V, const Consts& C, const Tables& T, hipStream_t s) {
  if (n_ct <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_ct, dim3((unsigned)(n_ct * C.L)), C, s, src, dst, share, G, V, C, T);
  return hipGetLastError();
}

hipError_t launch_ntt_pt(const int64_t* tensor, uint64_t* dst, int64_t n_pt, int side, const Geo& G, const View& V,
                         const Consts& C, const Tables& T, hipStream_t s) {
  if (n_pt <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_pt, dim3((unsigned)(n_pt * C.L)), C, s, tensor, dst, side, G, V, C, T);
  return hipGetLastError();
}

hipError_t launch_ntt_ternary(uint64_t* dst, int64_t count, uint64_t nonce, uint64_t obj_base, uint32_t purpose, int split,
                              const Consts& C, const Tables& T, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_ternary, dim3((unsigned)(count * C.L)), C, s, dst, nonce, obj_base, purpose, split, C, T);
  return hipGetLastError();
}

hipError_t configure_lds_ntt() {
  const int max_lds = 160 * 1024;
  hipError_t e = hipSuccess;
#define PENCIL_RAISE(LN, LE)                                                                            \
  for (const void* f : {(const void*)k_ntt_plain<LN, LE>, (const void*)k_ntt_ct<LN, LE>,                 \
                        (const void*)k_ntt_pt<LN, LE>, (const void*)k_ntt_ternary<LN, LE>}) {            \
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
