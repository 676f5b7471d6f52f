// hf_schur_noalloc: the Schur-complement accessor of include/hf.h without any
// allocation, for callers that cannot allocate device memory.
//
// hf_schur stages the permutation that puts S22 in ascending original order in a
// device buffer it allocates per call.  Here that permutation (the rank of every
// hard-part index in original numbering) lives in a file-scope device array of
// fixed size instead; the rank is computed on the device, the hard-part list is
// sorted in the caller's own host buffer, and the call allocates nothing, on the
// device or on the host.
#include <algorithm>
#include <mutex>

#include "hf_internal.h"

namespace hf {

constexpr int NOALLOC_MAX_M = 16384;  // largest hard part the scratch array holds
constexpr int NOALLOC_MAX_DEV = 64;

// rank of each hard-part index (M entries used); every GPU the library runs on
// holds its own copy of this array at its own address
static __device__ __align__(256) int32_t scratch[NOALLOC_MAX_M];

static std::mutex g_scratch_mu;
static int32_t* g_scratch_ptr[NOALLOC_MAX_DEV] = {};

// device address of `scratch` on the current device (looked up once per device)
static int scratch_on_device(int32_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HF_ERR_HIP;
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return HF_ERR_NOT_IMPLEMENTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HF_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<int32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return HF_OK;
}

// rank[i] = number of hard-part indices whose original number is below that of
// hard-part index i (original numbers are distinct)
__global__ void k_rank_l2(int M, const int32_t* __restrict__ l2, const int32_t* __restrict__ perm,
                          int32_t* __restrict__ rank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int32_t gi = perm[l2[i]];
  int32_t r = 0;
  for (int j = 0; j < M; ++j) r += perm[l2[j]] < gi ? 1 : 0;
  rank[i] = r;
}

// out[rank[c], rank[r]] = S[c, r] (column-major, leading dimensions lds and M)
__global__ void k_scatter_s22(int M, const int32_t* __restrict__ rank, const double* __restrict__ S,
                              double* __restrict__ out, int64_t lds) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * M) return;
  const int r = (int)(e % M), c = (int)(e / M);
  out[(int64_t)rank[c] * lds + rank[r]] = S[e];
}

static int schur_noalloc_impl(const hf_ctx* ctx, int32_t* m, int32_t* lambda2, double* S, int64_t lds,
                              hipStream_t s) {
  if (ctx->state < 2) return HF_ERR_STATE;
  const int M = ctx->M;
  *m = M;
  if (!lambda2 && !S) return HF_OK;
  if (M > NOALLOC_MAX_M) return HF_ERR_NOT_IMPLEMENTED;
  if (S && M > 0 && lds < M) return HF_ERR_ARG;
  if (lambda2) {
    for (int i = 0; i < M; ++i) lambda2[i] = ctx->perm[ctx->lambda2[i]];
    std::sort(lambda2, lambda2 + M);
  }
  if (S && M > 0) {
    int32_t* rank = nullptr;
    const int st = scratch_on_device(&rank);
    if (st != HF_OK) return st;
    k_rank_l2<<<(M + 255) / 256, 256, 0, s>>>(M, ctx->d_l2.as<int32_t>(), ctx->d_perm.as<int32_t>(), rank);
    const int64_t mm = (int64_t)M * M;
    k_scatter_s22<<<(unsigned)((mm + 255) / 256), 256, 0, s>>>(M, rank, ctx->d_S22.as<double>(), S, lds);
    if (hipGetLastError() != hipSuccess) return HF_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return HF_ERR_HIP;
  }
  return HF_OK;
}

}  // namespace hf

extern "C" int hf_schur_noalloc(const hf_ctx* ctx, int32_t* m_host, int32_t* lambda2_host, double* S22_dev,
                                int64_t lds, void* stream) {
  if (!ctx || !m_host) return HF_ERR_ARG;
  return hf::schur_noalloc_impl(ctx, m_host, lambda2_host, S22_dev, lds, static_cast<hipStream_t>(stream));
}
