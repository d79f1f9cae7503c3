// Setup of the paper-mode block-Jacobi preconditioner BJAC(k, t): eq. 3-1 with
// k outer steps, the block solve by t point-Jacobi sweeps inside each diagonal
// block (eq. 3-3), on contiguous row blocks of any size (Sec. 3.1; the paper
// runs one block per process). Nothing is inverted: the setup keeps an FP32
// copy of A's values, the reciprocals of the diagonal in FP64 and FP32, and
// each row's block column range; the application kernels live with the PCG
// kernels.
#include <algorithm>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace mpb {

__global__ __launch_bounds__(256) void poly_prep_kernel(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                                                        const double *val, const int32_t *blk_row, int nb,
                                                        float *val32, double *dinv64, float *dinv32, int32_t *rlo,
                                                        int32_t *rhi, int32_t *bad) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < nnz; i += stride) val32[i] = (float)val[i];
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += stride) {
    // block of row i: the last b with blk_row[b] <= i
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (blk_row[mid] <= i) lo = mid;
      else hi = mid;
    }
    rlo[i] = blk_row[lo];
    rhi[i] = blk_row[lo + 1];
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) d += val[k];
    if (!(d > 0.0)) {
      __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      d = 1.0;
    }
    const double r = 1.0 / d;
    dinv64[i] = r;
    dinv32[i] = (float)r;
  }
}

struct PolyLayout {
  int32_t *blk_row, *bad, *rlo, *rhi;
  float *val32, *dinv32;
  double *dinv64, *pbuf;
  size_t bytes;
};

static PolyLayout carve_poly(void *ws, int64_t n, int64_t nnz, int nb) {
  Carver c(ws);
  PolyLayout L{};
  L.blk_row = c.take<int32_t>(nb + 1);
  L.bad = c.take<int32_t>(1);
  L.rlo = c.take<int32_t>(n);
  L.rhi = c.take<int32_t>(n);
  L.val32 = c.take<float>(nnz);
  L.dinv32 = c.take<float>(n);
  L.dinv64 = c.take<double>(n);
  L.pbuf = c.take<double>(6 * n);
  L.bytes = c.used;
  return L;
}

static int check_poly(const bjac_csr *A, const int32_t *block_ptr, int32_t nb, const bjac_poly_params *pp) {
  if (!A || !block_ptr || !pp || nb < 1 || A->n < 1 || A->n >= ((int64_t)1 << 31) || A->nnz < 0) return BJAC_EINVAL;
  if (!A->row_ptr || !A->col_idx || !A->val) return BJAC_EINVAL;
  if (pp->k < 1 || pp->k > 64 || pp->t < 1 || pp->t > 64) return BJAC_EINVAL;
  if (pp->temporal < BJAC_TEMPORAL_NONE || pp->temporal > BJAC_TEMPORAL_LH) return BJAC_EINVAL;
  if (block_ptr[0] != 0 || block_ptr[nb] != A->n) return BJAC_EINVAL;
  for (int i = 0; i < nb; ++i)
    if (block_ptr[i + 1] <= block_ptr[i]) return BJAC_EINVAL;
  return BJAC_OK;
}

}  // namespace mpb

using namespace mpb;

extern "C" int bjac_poly_setup_query(const bjac_csr *A, const int32_t *block_ptr, int32_t nb,
                                     const bjac_poly_params *params, size_t *workspace_bytes) {
  if (!workspace_bytes) return BJAC_EINVAL;
  const int rc = check_poly(A, block_ptr, nb, params);
  if (rc) return rc;
  *workspace_bytes = carve_poly(nullptr, A->n, A->nnz, nb).bytes;
  return BJAC_OK;
}

extern "C" int bjac_poly_setup(const bjac_csr *A, const int32_t *block_ptr, int32_t nb,
                               const bjac_poly_params *params, void *workspace, size_t workspace_bytes, void *stream,
                               bjac_handle **out) {
  if (!out || !workspace) return BJAC_EINVAL;
  *out = nullptr;
  int rc = check_poly(A, block_ptr, nb, params);
  if (rc) return rc;
  const PolyLayout L = carve_poly(workspace, A->n, A->nnz, nb);
  if (L.bytes > workspace_bytes) return BJAC_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  MPB_HIP(hipMemcpyAsync(L.blk_row, block_ptr, sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, s));
  MPB_HIP(hipMemsetAsync(L.bad, 0, sizeof(int32_t), s));
  const int64_t work = std::max<int64_t>(A->n, A->nnz);
  const int G = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (work + 255) / 256));
  hipLaunchKernelGGL(poly_prep_kernel, dim3(G), dim3(256), 0, s, (int64_t)A->n, (int64_t)A->nnz, A->row_ptr,
                     A->col_idx, A->val, (const int32_t *)L.blk_row, (int)nb, L.val32, L.dinv64, L.dinv32, L.rlo,
                     L.rhi, L.bad);
  MPB_HIP(hipGetLastError());
  int32_t bad = 0;
  MPB_HIP(hipMemcpyAsync(&bad, L.bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPB_HIP(hipStreamSynchronize(s));
  if (bad) return BJAC_ENOTSPD;
  bjac_handle *h = new bjac_handle();
  h->kind = 1;
  h->n = A->n;
  h->nb = nb;
  h->stream = s;
  h->ws = (uint8_t *)workspace;
  h->ws_bytes = workspace_bytes;
  h->pk = params->k;
  h->pt = params->t;
  h->plow = params->low ? 1 : 0;
  h->prp = A->row_ptr;
  h->pci = A->col_idx;
  h->pval = A->val;
  h->pnnz = A->nnz;
  h->val32 = L.val32;
  h->dinv64 = L.dinv64;
  h->dinv32 = L.dinv32;
  h->rlo = L.rlo;
  h->rhi = L.rhi;
  h->pbuf = L.pbuf;
  h->blk_row = L.blk_row;
  h->policy.mode = h->plow ? BJAC_FIXED : BJAC_UNIFORM;
  h->policy.low = h->plow ? BJAC_FP32 : BJAC_FP64;
  h->policy.temporal = params->temporal;
  h->policy.adp_tol = params->adp_tol;
  h->h_blk_row.assign(block_ptr, block_ptr + nb + 1);
  h->h_tag_lo.assign(nb, (uint8_t)(h->plow ? BJAC_FP32 : BJAC_FP64));
  for (int i = 0; i < nb; ++i) h->max_block = std::max(h->max_block, block_ptr[i + 1] - block_ptr[i]);
  h->hist[h->plow ? BJAC_FP32 : BJAC_FP64] = nb;
  h->low_bytes = h->plow ? 4 * A->nnz + 4 * A->n : 8 * A->nnz + 8 * A->n;
  h->high_bytes = params->temporal ? 8 * A->nnz + 8 * A->n : 0;
  *out = h;
  return BJAC_OK;
}
