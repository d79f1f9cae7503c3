// Streaming probe: the HBM rate a plain kernel reaches for a given mix of
// read and write streams. Not a step of the method: it measures the practical
// ceiling the hot kernels' roofline fractions are read against (the SpMV and
// the fused update + application read several bytes for each one they write).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace mpb {

constexpr int kProbeMaxIn = 8, kProbeMaxOut = 2;
using f64x2 = double __attribute__((ext_vector_type(2)));

struct ProbePtrs {
  const double *in[kProbeMaxIn];
  double *out[kProbeMaxOut];
};

// Every lane moves U x 16 bytes per stream per step (U double2 loads in
// flight per stream), grid-stride; out[j] = (sum of the inputs) + j. The
// read-only mix writes one value per thread at the end so the loads are not
// dead. Loads and stores are non-temporal: every byte is touched once.
template <int NI, int NO, int U>
__global__ __launch_bounds__(256) void stream_kernel(ProbePtrs p, int64_t n2, double *sink) {
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256 * U;
  for (int64_t i0 = blockIdx.x * 256ll * U + threadIdx.x; i0 < n2; i0 += stride) {
    f64x2 s[U];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = f64x2{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NI; ++k)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + 256ll * u;
        if (i < n2) s[u] += __builtin_nontemporal_load((const f64x2 *)p.in[k] + i);
      }
#pragma unroll
    for (int j = 0; j < NO; ++j)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + 256ll * u;
        if (i < n2) __builtin_nontemporal_store(s[u] + (double)j, (f64x2 *)p.out[j] + i);
      }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += s[u].x + s[u].y;
  }
  if (NO == 0 && sink) sink[blockIdx.x * 256 + threadIdx.x] = acc;
}

template <int NI, int U>
static void launch_ni(int no, dim3 g, hipStream_t s, const ProbePtrs &p, int64_t n2, double *sink) {
  switch (no) {
    case 0: hipLaunchKernelGGL((stream_kernel<NI, 0, U>), g, dim3(256), 0, s, p, n2, sink); break;
    case 1: hipLaunchKernelGGL((stream_kernel<NI, 1, U>), g, dim3(256), 0, s, p, n2, sink); break;
    default: hipLaunchKernelGGL((stream_kernel<NI, 2, U>), g, dim3(256), 0, s, p, n2, sink); break;
  }
}

template <int U>
static void launch_u(int ni, int no, dim3 g, hipStream_t s, const ProbePtrs &p, int64_t n2, double *sink) {
  switch (ni) {
    case 0: launch_ni<0, U>(no, g, s, p, n2, sink); break;
    case 1: launch_ni<1, U>(no, g, s, p, n2, sink); break;
    case 2: launch_ni<2, U>(no, g, s, p, n2, sink); break;
    case 3: launch_ni<3, U>(no, g, s, p, n2, sink); break;
    case 4: launch_ni<4, U>(no, g, s, p, n2, sink); break;
    case 5: launch_ni<5, U>(no, g, s, p, n2, sink); break;
    case 6: launch_ni<6, U>(no, g, s, p, n2, sink); break;
    case 7: launch_ni<7, U>(no, g, s, p, n2, sink); break;
    default: launch_ni<8, U>(no, g, s, p, n2, sink); break;
  }
}

}  // namespace mpb

using namespace mpb;

extern "C" int bjac_stream_probe(const double *const *in, int32_t n_in, double *const *out, int32_t n_out,
                                 int64_t count, int32_t grid, int32_t unroll, double *sink, void *stream) {
  if (n_in < 0 || n_in > kProbeMaxIn || n_out < 0 || n_out > kProbeMaxOut || n_in + n_out < 1) return BJAC_EINVAL;
  if (count < 2 || (count & 1) || (n_in && !in) || (n_out && !out)) return BJAC_EINVAL;
  if (unroll != 1 && unroll != 2 && unroll != 4) return BJAC_EINVAL;
  ProbePtrs p{};
  for (int k = 0; k < n_in; ++k) {
    if (!in[k] || ((uintptr_t)in[k] & 15)) return BJAC_EINVAL;
    p.in[k] = in[k];
  }
  for (int j = 0; j < n_out; ++j) {
    if (!out[j] || ((uintptr_t)out[j] & 15)) return BJAC_EINVAL;
    p.out[j] = out[j];
  }
  if (n_out == 0 && !sink) return BJAC_EINVAL;   // the read-only mix needs grid * 256 doubles of sink
  const int64_t n2 = count / 2;
  int64_t G = grid > 0 ? grid : 8192;
  const int64_t need = (n2 + 256ll * unroll - 1) / (256ll * unroll);
  if (G > need) G = need;
  hipStream_t s = (hipStream_t)stream;
  const dim3 g((unsigned)G);
  if (unroll == 1) launch_u<1>(n_in, n_out, g, s, p, n2, sink);
  else if (unroll == 2) launch_u<2>(n_in, n_out, g, s, p, n2, sink);
  else launch_u<4>(n_in, n_out, g, s, p, n2, sink);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}
