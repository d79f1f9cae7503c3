// PCG hot path: q = A p fused with the p update and (p, q); the x / r update
// fused with the block-Jacobi application z = M^-1 r and the dots (r, r),
// (r, z); all scalars on the device, iterations replayed as HIP graphs.
// arXiv 2407.15973: Sec. 3.2 (PCG with M^-1_bjac), Algorithm 3.1 (fMP
// application), Algorithms 3.2 / 3.3 (adaptive switch), Sec. 4.2 (stopping
// test on the relative residual, x0 = 0).
//
// Work is split into wave tiles: each wave64 owns up to 64 consecutive rows
// (the SpMV) or up to 64 padded rows of whole diagonal blocks (the
// application) and runs every phase of its tile without workgroup barriers.
// A persistent grid of at most kMaxGrid workgroups walks the tiles
// round-robin over all its waves.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <type_traits>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace mpb {

// Wave tiles of a persistent grid, round-robin over every wave of the chip:
// wave w takes tiles w, w + W, w + 2W, ... (W waves), so at any moment the
// waves of all eight XCDs work on one window of consecutive rows. (Giving each
// XCD a contiguous eighth of the tiles instead, for the XCD's L2 to keep a
// row's neighbours a grid plane away, was slower on every workload measured:
// at 192^3 the FP16 application took 173 us against 165 us, the SpMV 159 us
// against 152 us.)
struct WaveIter {
  int t, step, end;
  __device__ explicit WaveIter(int T) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    t = (int)blockIdx.x * 4 + wv;
    step = (int)gridDim.x * 4;
    end = T;
  }
};

// Workgroups of a persistent grid for T wave tiles: no more than one resident
// round of the kernel (occupancy x compute units), at most kGridPerCu per
// compute unit, at least one tile per wave (on a 64 x 64 Poisson problem, 64
// tiles, one tile per wave instead of two cut the iteration from 21.5 to
// 18.3 us: the tiles spread over twice the compute units), a multiple of 8
// when possible.
static int grid_for_waves(int T, const void *kernel, int per_cu_max = kGridPerCu) {
  // occupancy and compute units per (kernel, device), queried once under a
  // lock, so handles used from several threads (or devices) share the cache
  static std::mutex mu;
  static std::map<std::pair<const void *, int>, std::pair<int, int>> cap;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  std::pair<int, int> pc;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cap.find({kernel, dev});
    if (it == cap.end()) {
      int per_cu = 0, cus = 0;
      if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1 ||
          cus < 1) {
        per_cu = 1;
        cus = 256;
      }
      it = cap.emplace(std::make_pair(kernel, dev), std::make_pair(per_cu, cus)).first;
    }
    pc = it->second;
  }
  const int resident = std::min(pc.first, per_cu_max) * pc.second;
  int G = (T + 3) / 4;
  if (G > resident) G = resident;
  if (G > kMaxGrid) G = kMaxGrid;
  if (G >= 8) G &= ~7;
  return G < 1 ? 1 : G;
}

// LDS written by one lane and read by another lane of the same wave: the
// hardware keeps a wave's LDS operations in order; this keeps the compiler
// from moving them across the exchange point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over a 256-thread workgroup; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Cross-workgroup reduction without cache maintenance. Each workgroup
// publishes its partial with a device-scope atomic store into a slot that
// holds kEmpty, then takes a ticket with a device-scope atomic add; device-
// scope atomics are coherent across the XCDs' L2 caches, so no write-back or
// invalidate fence is needed. The workgroup with the last ticket reads every
// slot with device-scope atomic loads, waiting for slots whose store is still
// in flight (every writer issued its store before its ticket, so the wait
// ends; kSpinCap bounds it regardless), and resets each slot to kEmpty for the
// next launch. kEmpty is a signalling-NaN pattern that no arithmetic result
// can take (arithmetic only produces quiet NaNs).
constexpr uint64_t kEmpty = 0x7FF4D1CE0000BEEFull;
constexpr int kSpinCap = 1 << 22;

__device__ __forceinline__ void publish(double *slot, double v) {
  __hip_atomic_store((uint64_t *)slot, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in every thread of the workgroup that took the last ticket.
__device__ __forceinline__ bool last_workgroup(uint32_t *ticket, int *sh_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *sh_flag = (t == gridDim.x - 1);
  }
  __syncthreads();
  return *sh_flag != 0;
}

// Deterministic fixed-order sums of NS interleaved sets of n published
// partials (partial i of set s at p[i * stride + s]) by the last workgroup;
// results valid in thread 0. ok_out (thread 0) turns false if a slot never
// filled. Every thread first issues the loads of all its slots (at most
// kMaxGrid / 256 per set; indices past n re-read slot n - 1 and are ignored),
// so the collection costs one memory round trip rather than one per slot;
// only slots still empty are polled again.
template <int NS>
__device__ __forceinline__ void sum_partials_n(double *p, int n, int stride, double *sh, int *ok_out,
                                               double (&out)[NS]) {
  constexpr int K = kMaxGrid / 256;
  uint64_t u[K][NS];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = min((int)threadIdx.x + 256 * k, n - 1);
#pragma unroll
    for (int q = 0; q < NS; ++q)
      u[k][q] = __hip_atomic_load((uint64_t *)(p + (int64_t)i * stride + q), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  }
  double acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.0;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = (int)threadIdx.x + 256 * k;
    if (i < n) {
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        double *slot = p + (int64_t)i * stride + q;
        uint64_t v = u[k][q];
        int spins = 0;
        while (v == kEmpty && ++spins < kSpinCap)
          v = __hip_atomic_load((uint64_t *)slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = ok && v != kEmpty;
        __hip_atomic_store((uint64_t *)slot, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        acc[q] += __longlong_as_double((long long)v);
      }
    }
  }
  if (!ok) atomicAnd(ok_out, 0);
#pragma unroll
  for (int q = 0; q < NS; ++q) out[q] = block_sum(acc[q], sh);
}

__device__ __forceinline__ double sum_partials(double *p, int n, int stride, double *sh, int *ok_out) {
  double out[1];
  sum_partials_n<1>(p, n, stride, sh, ok_out, out);
  return out[0];
}

static_assert(offsetof(PcgState, cidx) == offsetof(PcgState, status) + 4 && offsetof(PcgState, status) % 8 == 0,
              "status and cidx are read as one 8-byte word");

// The 16-bit row-relative copy of A's column indices (col - row) read by the
// PCG SpMVs; any entry farther than 32767 rows from its row clears *flag, and
// the products keep the 32-bit indices.
__global__ __launch_bounds__(256) void off16_kernel(int n, const int32_t *rp, const int32_t *ci, int16_t *o,
                                                    int32_t *flag) {
  bool ok = true;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int d = ci[k] - i;
      ok = ok && d >= -32768 && d <= 32767;
      o[k] = (int16_t)d;
    }
  }
  if (!ok) __hip_atomic_store(flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 8-bit codes of the column offsets. Structured matrices have a handful of
// distinct offsets col - row (7 for a 7-point stencil), so a 256-entry
// dictionary of them lets every entry's column be stored in one byte: the
// code is the offset's slot in an open-addressing table (multiplicative hash,
// linear probing). The table is built per workgroup in LDS (a read before
// every compare-and-swap, so the few hot slots are rarely written) and merged
// into the global table; more than 256 distinct offsets set *overflow.
constexpr int kDictSize = 256;
constexpr int kDictEmpty = (int)0x80000000;   // no offset col - row of an int32 CSR takes this value

__device__ __forceinline__ unsigned dict_hash(int d) { return ((unsigned)d * 2654435761u) >> 24; }

template <bool GLOBAL>
__device__ __forceinline__ bool dict_insert(int *tab, int d) {
  unsigned h = dict_hash(d);
  for (int probe = 0; probe < kDictSize; ++probe, h = (h + 1) & (kDictSize - 1)) {
    const int cur = GLOBAL ? __hip_atomic_load(tab + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : __hip_atomic_load(tab + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == d) return true;
    if (cur == kDictEmpty) {
      const int old = atomicCAS(tab + h, kDictEmpty, d);
      if (old == kDictEmpty || old == d) return true;
    }
  }
  return false;
}

__global__ __launch_bounds__(256) void dict_fill_kernel(int *gtab, int *overflow) {
  gtab[threadIdx.x] = kDictEmpty;
  if (threadIdx.x == 0) *overflow = 0;
}

__global__ __launch_bounds__(256) void dict_build_kernel(int n, const int32_t *rp, const int32_t *ci, int *gtab,
                                                         int *overflow) {
  __shared__ int tab[kDictSize];
  __shared__ int ovf;
  tab[threadIdx.x] = kDictEmpty;
  if (threadIdx.x == 0) ovf = 0;
  __syncthreads();
  bool ok = true;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n && ok; i += gridDim.x * 256)
    for (int k = rp[i]; k < rp[i + 1] && ok; ++k) ok = dict_insert<false>(tab, ci[k] - i);
  if (!ok) ovf = 1;
  __syncthreads();
  const int d = tab[threadIdx.x];
  if (!ovf && d != kDictEmpty && !dict_insert<true>(gtab, d)) ovf = 1;
  __syncthreads();
  if (threadIdx.x == 0 && ovf) __hip_atomic_store(overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The compact copy of A's column structure the PCG SpMVs read: the 8-bit
// codes when the dictionary holds every offset (*cidx = 2), else the 16-bit
// offsets col - row when all fit (*cidx stays 1), else none (*cidx = 0).
// o8 and o16 share the workspace region.
__global__ __launch_bounds__(256) void idx_encode_kernel(int n, const int32_t *rp, const int32_t *ci, const int *gtab,
                                                         const int *overflow, uint8_t *o8, int16_t *o16,
                                                         int32_t *cidx) {
  __shared__ int tab[kDictSize];
  tab[threadIdx.x] = gtab[threadIdx.x];
  __syncthreads();
  if (*overflow == 0) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int d = ci[k] - i;
        unsigned h = dict_hash(d);
        // present: the build inserted every offset (the probe count is bounded all the same)
        for (int probe = 0; probe < kDictSize && tab[h] != d; ++probe) h = (h + 1) & (kDictSize - 1);
        o8[k] = (uint8_t)h;
      }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) __hip_atomic_store(cidx, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  bool ok = true;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int d = ci[k] - i;
      ok = ok && d >= -32768 && d <= 32767;
      o16[k] = (int16_t)d;
    }
  }
  if (!ok) __hip_atomic_store(cidx, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 8-bit codes of the matrix values (a value dictionary, as in CSR-VI, Kourtis,
// Goumas and Koziris 2008). Matrices of PDEs with piecewise-constant
// coefficients hold few distinct values (17 on the 192^3 held-out problem),
// so with 8-bit column codes as well an entry takes 2 bytes instead of 9.
// The table is keyed by the value's 64 bits (exact: +0 and -0, and every NaN
// pattern, are distinct keys); a value equal to the empty key, or more than
// 256 distinct values, set *overflow and the products read the 8-byte values.
constexpr uint64_t kVDictEmpty = 0x7FF4DEADBEEF0001ull;   // a signalling NaN pattern

__device__ __forceinline__ unsigned vdict_hash(uint64_t b) { return (unsigned)((b * 0x9E3779B97F4A7C15ull) >> 56); }

template <bool GLOBAL>
__device__ __forceinline__ bool vdict_insert(unsigned long long *tab, unsigned long long b) {
  if (b == kVDictEmpty) return false;
  unsigned h = vdict_hash(b);
  for (int probe = 0; probe < kDictSize; ++probe, h = (h + 1) & (kDictSize - 1)) {
    const unsigned long long cur = GLOBAL ? __hip_atomic_load(tab + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                          : __hip_atomic_load(tab + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == b) return true;
    if (cur == kVDictEmpty) {
      const unsigned long long old = atomicCAS(tab + h, (unsigned long long)kVDictEmpty, b);
      if (old == kVDictEmpty || old == b) return true;
    }
  }
  return false;
}

__global__ __launch_bounds__(256) void vdict_fill_kernel(unsigned long long *gtab, int *overflow) {
  gtab[threadIdx.x] = kVDictEmpty;
  if (threadIdx.x == 0) *overflow = 0;
}

__global__ __launch_bounds__(256) void vdict_build_kernel(int64_t nnz, const double *v, unsigned long long *gtab,
                                                          int *overflow) {
  __shared__ unsigned long long tab[kDictSize];
  __shared__ int ovf;
  tab[threadIdx.x] = kVDictEmpty;
  if (threadIdx.x == 0) ovf = 0;
  __syncthreads();
  bool ok = true;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz && ok; k += (int64_t)gridDim.x * 256)
    ok = vdict_insert<false>(tab, (unsigned long long)__double_as_longlong(v[k]));
  if (!ok) ovf = 1;
  __syncthreads();
  const unsigned long long b = tab[threadIdx.x];
  if (!ovf && b != kVDictEmpty && !vdict_insert<true>(gtab, b)) ovf = 1;
  __syncthreads();
  if (threadIdx.x == 0 && ovf) __hip_atomic_store(overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The value codes, when the dictionary holds every value and the column
// structure is 8-bit coded (*cidx == 2); vcode_commit_kernel then raises
// *cidx to 3 (a launch of its own: every workgroup here reads *cidx first).
__global__ __launch_bounds__(256) void val_encode_kernel(int64_t nnz, const double *v,
                                                         const unsigned long long *gtab, const int *overflow,
                                                         uint8_t *v8, const int32_t *cidx) {
  __shared__ unsigned long long tab[kDictSize];
  tab[threadIdx.x] = gtab[threadIdx.x];
  __syncthreads();
  if (*overflow != 0 || *cidx != 2) return;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * 256) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v[k]);
    unsigned h = vdict_hash(b);
    // present: the build inserted every value (the probe count is bounded all the same)
    for (int probe = 0; probe < kDictSize && tab[h] != b; ++probe) h = (h + 1) & (kDictSize - 1);
    v8[k] = (uint8_t)h;
  }
}

__global__ void vcode_commit_kernel(const int *overflow, int32_t *cidx) {
  if (*overflow == 0 && *cidx == 2) *cidx = 3;
}

__global__ __launch_bounds__(256) void fill_empty_kernel(double *p, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) ((uint64_t *)p)[i] = kEmpty;
}

// ------------------------------------------------------------------- SpMV
// SPMV_CG: the single-reduction iteration's product w = A u (u gathered at
// the neighbours, no p update) with the three dots (r, r), (r, u), (w, u).
enum SpmvMode { SPMV_PLAIN = 0, SPMV_PCG = 1, SPMV_CG = 2 };

struct SpmvArgs {
  int32_t n, ntiles;
  const int32_t *rp, *ci;
  const double *v;
  const double *z;      // PCG: preconditioned residual; PLAIN: the vector p; CG: u = M^-1 r
  const double *rv;     // CG: the residual r (read at the row only)
  const double *pold;
  double *pnew, *q;
  PcgState *st;
  double *part;
  const int16_t *o16;   // PCG / CG: col - row of every entry (st->cidx == 1), or its 8-bit code
                        // (st->cidx == 2: the same region read as bytes)
  const int *dict;      // the codes' dictionary: offset of code c at dict[c]
  const uint8_t *v8;    // st->cidx == 3: the 8-bit value codes (16-byte aligned)
  const double *vdict;  // st->cidx == 3: value of code c at vdict[c]
  int32_t nnz8;         // nnz rounded down to a multiple of 8: whole 16-byte chunks of every array
  int32_t nnz16;        // nnz rounded down to a multiple of 16 (8-bit codes: 16 per chunk)
  int32_t vec;          // values and indices 16-byte aligned: tiles may be staged in 16-byte chunks
};

// Column index modes of the SpMV tiles: the CSR's 32-bit indices, 16-bit
// offsets col - row, 8-bit codes of col - row; IX8V: 8-bit codes of col - row
// and 8-bit codes of the values.
enum IdxMode { IX32 = 0, IX16 = 1, IX8 = 2, IX8V = 3 };
template <int IX>
using IdxT = std::conditional_t<IX == IX32, int32_t, std::conditional_t<IX == IX16, int16_t, uint8_t>>;

// Dot product of one CSR row with p_new = z + beta p_old (the p update of PCG
// folded into the product; PLAIN mode reads p = z). Seven entries at a time
// (a 7-point row in one group: measured 52.6 -> 50.7 us per product at 128^3
// against groups of eight, whose clamped eighth gather is pure overhead there)
// with every load in flight before the first multiply: indices past the row
// end are clamped to its last entry and their values replaced by zero, so
// there is no branch inside a group. Also returns p_new of the row itself
// when the row stores its diagonal.
template <bool PCG, int IX, bool FIND = PCG>
__device__ __forceinline__ double row_dot(const double *__restrict__ z, const double *__restrict__ pold,
                                          const IdxT<IX> *__restrict__ cidx, const void *__restrict__ vals,
                                          double beta, int base, int len, int row, double &prow, bool &found,
                                          const int *dict, const double *vdict) {
  constexpr int U = 7;
  double acc = 0.0;
  for (int k0 = 0; k0 < len; k0 += U) {
    int cs[U];
    double vs[U], g[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int idx = base + min(k0 + k, len - 1);
      if constexpr (IX == IX32) cs[k] = cidx[idx];
      else if constexpr (IX == IX16) cs[k] = (int)cidx[idx] + row;
      else cs[k] = dict[cidx[idx]] + row;
      double v;
      if constexpr (IX == IX8V) v = vdict[((const uint8_t *)vals)[idx]];
      else v = ((const double *)vals)[idx];
      vs[k] = (k0 + k < len) ? v : 0.0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) g[k] = PCG ? fma(beta, pold[cs[k]], z[cs[k]]) : z[cs[k]];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      acc = fma(vs[k], g[k], acc);
      if (FIND && cs[k] == row) {
        prow = g[k];
        found = true;
      }
    }
  }
  return acc;
}

// s_waitcnt operand that waits for every vector memory operation and leaves the
// other counters free (gfx9 encoding: vmcnt 0, expcnt 7, lgkmcnt 15)
constexpr int kVmcntZero = 0x0F70;

using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
using u32x2 = unsigned int __attribute__((ext_vector_type(2)));

// Cache hints of the streaming solves (NT = true): non-temporal loads and
// stores for data that one launch touches once, when the bytes of an
// iteration are far beyond what the last-level cache can keep from one
// iteration to the next; plain accesses otherwise.
template <bool NT, class T>
__device__ __forceinline__ T ld_hint(const T *p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void st_hint(T v, T *p) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// The tiles of one wave; returns the wave's partial (p_new, q). REL: the
// column indices are the 16-bit row-relative copy (one loop per choice,
// decided once per launch).
//
// A tile's CSR entries are staged into the wave's LDS slice in whole 16-byte
// chunks from the 8-entry boundary at or below its first entry: 4 loads of
// values and 1 (16-bit) or 2 (32-bit) of indices per lane instead of one load
// per entry and array. Tiles whose window would pass the last whole 8-entry
// group of the arrays, or that hold more than a slice, read their rows from
// memory unstaged. The matrix is read once per product: non-temporal loads keep
// it from displacing the vectors, which the next kernel then finds in the
// last-level cache.
//
// Software-pipelined by one tile: tile t+1's chunk loads are issued before
// tile t's gathers of z and p_old, so the two round trips overlap (the row
// pointers run two tiles ahead), and the q / p_new stores of tile t are held
// back until after tile t+1's loads are issued.
struct Dots3 {
  double a = 0.0, b = 0.0, c = 0.0;
};

template <int SM, int IX, bool NT>
__device__ __forceinline__ Dots3 spmv_tiles(const SpmvArgs &a, double beta, double *sv, int *sc, const int *dict,
                                            const double *vdict) {
  constexpr bool PCG = SM == SPMV_PCG;   // p = z + beta p_old gathered, (p, q)
  constexpr bool CG = SM == SPMV_CG;     // u gathered, (r, r), (r, u), (w, u)
  constexpr bool VC = IX == IX8V;        // 8-bit value codes in place of the values
  constexpr int SLOT = kSpmvSlot;
  using IT = IdxT<IX>;
  constexpr int VB = VC ? 1 : 8;                                       // bytes per value
  constexpr int NV = (SLOT * VB + 16 * 64 - 1) / 16 / 64;             // value chunks per lane
  constexpr int NC = (SLOT * (int)sizeof(IT) + 16 * 64 - 1) / 16 / 64;  // index chunks per lane
  constexpr int EV = 16 / VB, EC = 16 / (int)sizeof(IT);              // entries per chunk
  constexpr int GA = EC > 8 ? EC : 8;                                 // window alignment (entries)
  const int32_t *__restrict__ rp = a.rp;
  const IT *__restrict__ cix = IX == IX32 ? (const IT *)a.ci : (const IT *)a.o16;
  const double *__restrict__ vv_g = a.v;
  const double *__restrict__ z = a.z;
  const double *__restrict__ pold = a.pold;
  const IT *sci = (const IT *)sc;
  const int lane = threadIdx.x & 63;
  Dots3 dot;
  bool s_has = false;   // q and p_new of the previous tile, stored after the next loads
  int s_row = 0;
  double s_q = 0.0, s_p = 0.0;
  WaveIter it(a.ntiles);
  // row pointers of a lane's row in tile t (row clamped into the tile); tiles
  // at or past the wave's end are not read
  auto fetch_rp = [&](int t, int &s_out, int &e_out) {
    s_out = e_out = 0;
    if (t < it.end) {
      const int rc = min(t * 64 + lane, min(a.n, t * 64 + 64) - 1);
      s_out = rp[rc];
      e_out = rp[rc + 1];
    }
  };
  // staging window of tile t: chunk-aligned base and entries from there to
  // the tile's end (0: the tile is read unstaged)
  auto window = [&](int t, int s, int e, int &base, int &need) {
    const int e0 = __builtin_amdgcn_readlane(s, 0);
    const int last = min(a.n, t * 64 + 64) - 1 - t * 64;
    const int cnt = t < it.end ? __builtin_amdgcn_readlane(e, last) - e0 : 0;
    base = e0 & ~(GA - 1);
    need = e0 - base + cnt;
    // every chunk read starts below base + need and lies below base + need
    // rounded up to GA entries, which must not pass the last whole group
    if (!a.vec || cnt <= 0 || need > SLOT || base + ((need + GA - 1) & ~(GA - 1)) > (GA == 8 ? a.nnz8 : a.nnz16))
      need = 0;
  };
  auto stage = [&](int base, int need, u32x4 (&gv)[NV], u32x4 (&gc)[NC]) {
    const u32x4 zero = {0u, 0u, 0u, 0u};
    const u32x4 *vp = VC ? (const u32x4 *)(a.v8 + base) : (const u32x4 *)(vv_g + base);
    const u32x4 *cp = (const u32x4 *)(cix + base);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int c = lane + 64 * q;
      gv[q] = c * EV < need ? __builtin_nontemporal_load(vp + c) : zero;
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int c = lane + 64 * q;
      gc[q] = c * EC < need ? __builtin_nontemporal_load(cp + c) : zero;
    }
  };
  int s_c, e_c, s_n, e_n, base_c, need_c;
  u32x4 gv[NV], gc[NC];
  fetch_rp(it.t, s_c, e_c);
  fetch_rp(it.t + it.step, s_n, e_n);
  window(it.t, s_c, e_c, base_c, need_c);
  stage(base_c, need_c, gv, gc);
  // the first tile's chunks in registers before the loop: inside it the
  // compiler then needs no wait on the loads of the tile after
  __builtin_amdgcn_s_waitcnt(kVmcntZero);
  for (; it.t < it.end; it.t += it.step) {
    const int tn = it.t + it.step;
    int s_nn, e_nn, base_n, need_n;
    fetch_rp(tn + it.step, s_nn, e_nn);
    window(tn, s_n, e_n, base_n, need_n);
    u32x4 hv[NV], hc[NC];
    stage(base_n, need_n, hv, hc);
    if (s_has) {
      st_hint<NT>(s_q, a.q + s_row);
      if (PCG) st_hint<NT>(s_p, a.pnew + s_row);
      s_has = false;
    }
    const int row = it.t * 64 + lane;
    const bool has = row < a.n;
    const int len = has ? e_c - s_c : 0;
    double acc = 0.0, prow = 0.0;
    bool found = false;
    const double rrow = CG ? a.rv[min(row, a.n - 1)] : 0.0;   // in flight with the gathers
    if (need_c > 0) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const int c = lane + 64 * q;
        if (c * EV < need_c) ((u32x4 *)sv)[c] = gv[q];
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int c = lane + 64 * q;
        if (c * EC < need_c) ((u32x4 *)sc)[c] = gc[q];
      }
      wave_lds_sync();
      acc = row_dot<PCG, IX, PCG || CG>(z, pold, sci, sv, beta, s_c - base_c, len, row, prow, found, dict, vdict);
      wave_lds_sync();
    } else {
      acc = row_dot<PCG, IX, PCG || CG>(z, pold, cix, VC ? (const void *)a.v8 : (const void *)vv_g, beta, s_c, len,
                                        row, prow, found, dict, vdict);
    }
    s_has = has;
    s_row = row;
    s_q = acc;
    if (has && PCG) {
      const double pr = found ? prow : fma(beta, pold[row], z[row]);
      s_p = pr;
      dot.a = fma(pr, acc, dot.a);
    }
    if (has && CG) {
      const double ur = found ? prow : z[row];
      dot.a = fma(rrow, rrow, dot.a);
      dot.b = fma(rrow, ur, dot.b);
      dot.c = fma(acc, ur, dot.c);
    }
    s_c = s_n;
    e_c = e_n;
    s_n = s_nn;
    e_n = e_nn;
    base_c = base_n;
    need_c = need_n;
#pragma unroll
    for (int q = 0; q < NV; ++q) gv[q] = hv[q];
#pragma unroll
    for (int q = 0; q < NC; ++q) gc[q] = hc[q];
  }
  if (s_has) {
    st_hint<NT>(s_q, a.q + s_row);
    if (PCG) st_hint<NT>(s_p, a.pnew + s_row);
  }
  return dot;
}

// State transition of the single-reduction iteration, after w = A u and the
// dots (r, r), (r, u), (w, u) of the residual r the last update left (the
// Chronopoulos-Gear recurrence): convergence test on r (the iteration count
// is the number of x updates, as in the textbook form), then
// beta = gamma / gamma_old and alpha = gamma / (delta - beta gamma / alpha_old)
// (beta = 0, alpha = gamma / delta for the first direction or after a
// restart) for the next update.
__device__ __forceinline__ void cg_after_spmv(PcgState *st, double rr, double gamma, double delta) {
  st->rr = rr;
  if (st->restart) {
    st->relres = sqrt(rr) / st->rnorm0;
  } else if (st->iter < 0) {
    st->rnorm0 = sqrt(rr);
    st->iter = 0;
    st->relres = INFINITY;
    if (st->rnorm0 == 0.0) {
      st->relres = 0.0;
      st->status = ST_CONVERGED;
      return;
    }
  } else {
    st->iter += 1;
    st->relres = sqrt(rr) / st->rnorm0;
    if (st->relres_hist) st->relres_hist[st->iter - 1] = st->relres;
    if (st->relres <= st->tol) {
      st->status = ST_CONVERGED;
      return;
    }
  }
  st->rz = gamma;
  if (!(gamma > 0.0)) {
    st->status = ST_BREAKDOWN;
    return;
  }
  const bool first = st->iter == 0 || st->restart;
  const double beta = first ? 0.0 : gamma / st->rho;
  const double denom = first ? delta : delta - beta * gamma / st->alpha;
  st->pq = denom;   // (p, A p) of the new direction in exact arithmetic
  if (!(denom > 0.0)) {
    st->status = ST_BREAKDOWN;
    return;
  }
  st->beta = beta;
  st->alpha = gamma / denom;
  st->rho = gamma;
  st->restart = 0;
  if (st->iter >= st->maxit) st->status = ST_MAXIT;
}

template <int SM, bool NT = false>
__global__ __launch_bounds__(256) void spmv_kernel(SpmvArgs a) {
  constexpr bool PCG = SM == SPMV_PCG;
  constexpr bool CG = SM == SPMV_CG;
  constexpr int SLOT = kSpmvSlot;
  __shared__ __align__(16) double svs[4][SLOT];
  __shared__ __align__(16) int scs[4][SLOT];
  __shared__ double sh[4];
  __shared__ int flag, ok;
  __shared__ int sdict[kDictSize];
  __shared__ double svdict[kDictSize];
  // status and cidx are adjacent: one load before the early exit
  int2 sr = make_int2(ST_RUNNING, 0);
  if (PCG || CG) sr = *(const int2 *)&a.st->status;
  if ((PCG || CG) && sr.x != ST_RUNNING) return;
  const double beta = PCG ? a.st->beta : 0.0;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ix = (PCG || CG) && a.o16 ? sr.y : IX32;   // uniform over the grid
  Dots3 dot;
  if constexpr (PCG || CG) {
    if (ix == IX8V) {
      sdict[threadIdx.x] = a.dict[threadIdx.x];
      svdict[threadIdx.x] = a.vdict[threadIdx.x];
      __syncthreads();
      dot = spmv_tiles<SM, IX8V, NT>(a, beta, svs[wv], scs[wv], sdict, svdict);
    } else if (ix == IX8) {
      sdict[threadIdx.x] = a.dict[threadIdx.x];
      __syncthreads();
      dot = spmv_tiles<SM, IX8, NT>(a, beta, svs[wv], scs[wv], sdict, svdict);
    } else if (ix == IX16) {
      dot = spmv_tiles<SM, IX16, NT>(a, beta, svs[wv], scs[wv], sdict, svdict);
    } else {
      dot = spmv_tiles<SM, IX32, NT>(a, beta, svs[wv], scs[wv], sdict, svdict);
    }
  } else {
    dot = spmv_tiles<SPMV_PLAIN, IX32, NT>(a, beta, svs[wv], scs[wv], sdict, svdict);
  }
  if constexpr (PCG) {
    const double bs = block_sum(dot.a, sh);
    if (threadIdx.x == 0) {
      publish(a.part + blockIdx.x, bs);
      ok = 1;
    }
    if (last_workgroup(&a.st->ticket_a, &flag)) {
      const double pq = sum_partials(a.part, gridDim.x, 1, sh, &ok);
      if (threadIdx.x == 0) {
        PcgState *st = a.st;
        st->pq = pq;
        if (!ok) {
          st->status = ST_SYNC_FAIL;
        } else if (!(pq > 0.0)) {
          st->status = ST_BREAKDOWN;
        } else {
          st->alpha = st->rho / pq;
        }
        __hip_atomic_store(&st->ticket_a, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  } else if constexpr (CG) {
    const double b0 = block_sum(dot.a, sh);
    const double b1 = block_sum(dot.b, sh);
    const double b2 = block_sum(dot.c, sh);
    if (threadIdx.x == 0) {
      publish(a.part + 3 * blockIdx.x, b0);
      publish(a.part + 3 * blockIdx.x + 1, b1);
      publish(a.part + 3 * blockIdx.x + 2, b2);
      ok = 1;
    }
    if (last_workgroup(&a.st->ticket_a, &flag)) {
      double t[3];
      sum_partials_n<3>(a.part, gridDim.x, 3, sh, &ok, t);
      if (threadIdx.x == 0) {
        PcgState *st = a.st;
        if (!ok) st->status = ST_SYNC_FAIL;
        else cg_after_spmv(st, t[0], t[1], t[2]);
        __hip_atomic_store(&st->ticket_a, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// ------------------------------------------------- block-Jacobi application
// Launch modes: x/r update fused with the application (PCG), update only
// (adaptive switch, first half), application of the map the device-side
// switch chose (second half), standalone application z = M^-1 rin.
// M_CG: the single-reduction (Chronopoulos-Gear) iteration: p = u + beta p,
// s = w + beta s, x += alpha p, r -= alpha s, then u = M^-1 r, with no
// reduction (the dots are taken by the following SpMV).
enum ApplyMode { M_FUSED = 0, M_UPD = 1, M_APPDEV = 2, M_APP = 3, M_CG = 4 };

struct ApplyArgs {
  int32_t ntiles, nb, n, want_high;
  const int32_t *tile_blk, *blk_row;
  const uint8_t *bpad;
  DevMap map;
  int64_t off0;  // fast path: block k of the map starts at base + off0 + k * B^2 * bytes
  double *x, *r, *z;
  const double *p, *q, *rin;
  PcgState *st;
  double *part;
  double *pw, *sw;   // M_CG: p and s = A p, read and written in place (z holds u, q holds w = A u)
};

// The fragment one lane holds of one 16-row tile of a stored block, and its
// contribution to z: lane l owns row l % 16 and the columns congruent to
// l / 16 mod 4; the four column classes are summed across lanes at the end.
template <int B, int P>
struct Frag {
  static constexpr int K = B / 4;
  static constexpr int BY = prec_bytes(P);
  static constexpr int V = 16 / BY;
  static constexpr int G = (K + V - 1) / V;
  uint4 h[G];

  // NT: non-temporal loads (streaming solves, where the stored inverses
  // cannot stay in the last-level cache from one iteration to the next)
  template <bool NT = false>
  __device__ __forceinline__ void load(const uint8_t *blk, int mt, int lane) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int vg = layout_vg(B, V, g);
      const uint8_t *src = blk + (layout_group_base(B, V, mt, g) + (int64_t)lane * vg) * BY;
      if (vg * BY == 16) {
        const u32x4 t = NT ? __builtin_nontemporal_load((const u32x4 *)src) : *(const u32x4 *)src;
        h[g] = make_uint4(t.x, t.y, t.z, t.w);
      } else {
        const u32x2 t = NT ? __builtin_nontemporal_load((const u32x2 *)src) : *(const u32x2 *)src;
        h[g] = make_uint4(t.x, t.y, 0u, 0u);
      }
    }
  }

  // sum over this lane's columns, then over the four column classes; the row
  // total is valid in lanes 0..15
  __device__ __forceinline__ double dot(const float *r32, const double *r64, int lane) const {
    const int kq = lane >> 4;
    if constexpr (P == P64) {
      double acc = 0.0;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        acc = fma(__hiloint2double((int)h[g].y, (int)h[g].x), r64[4 * (2 * g) + kq], acc);
        acc = fma(__hiloint2double((int)h[g].w, (int)h[g].z), r64[4 * (2 * g + 1) + kq], acc);
      }
      acc += __shfl_xor(acc, 16, kWave);
      acc += __shfl_xor(acc, 32, kWave);
      return acc;
    } else {
      float acc = 0.0f;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int vg = layout_vg(B, V, g);
        const uint32_t w[4] = {h[g].x, h[g].y, h[g].z, h[g].w};
#pragma unroll
        for (int e = 0; e < V; ++e) {
          if (e < vg) {
            float hv;
            if constexpr (P == P32) hv = __uint_as_float(w[e]);
            else if constexpr (P == PBF16) hv = (e & 1) ? bf16_hi(w[e >> 1]) : bf16_lo(w[e >> 1]);
            else hv = (e & 1) ? f16_hi(w[e >> 1]) : f16_lo(w[e >> 1]);
            acc = fmaf(hv, r32[4 * (g * V + e) + kq], acc);
          }
        }
      }
      acc += __shfl_xor(acc, 16, kWave);
      acc += __shfl_xor(acc, 32, kWave);
      return (double)acc;
    }
  }

  // this lane's entry of k-step KS (column 4 KS + lane / 16 of its row), in
  // the accumulation type: double for FP64, float for the others
  template <int KS>
  __device__ __forceinline__ auto value() const {
    constexpr int g = KS / V, e = KS % V;
    if constexpr (P == P64) {
      if constexpr (e == 0) return __hiloint2double((int)h[g].y, (int)h[g].x);
      else return __hiloint2double((int)h[g].w, (int)h[g].z);
    } else {
      constexpr int c = P == P32 ? e : e >> 1;
      const uint32_t w = c == 0 ? h[g].x : c == 1 ? h[g].y : c == 2 ? h[g].z : h[g].w;
      if constexpr (P == P32) return __uint_as_float(w);
      else if constexpr (P == PBF16) return (e & 1) ? bf16_hi(w) : bf16_lo(w);
      else return (e & 1) ? f16_hi(w) : f16_lo(w);
    }
  }
};

// Sum over the 16 lanes of a DPP row, left in every lane of the row: pairs
// within quads, then quads (quad permutations), then half-rows (half-row
// mirror), then the two halves (row mirror). Each step adds the same two
// partial sums in every lane of a pair, so all 16 lanes hold the same value.
__device__ __forceinline__ int dpp_row_step(int v, int step) {
  switch (step) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    default: return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false); // row_mirror
  }
}
__device__ __forceinline__ float row16_sum(float v) {
#pragma unroll
  for (int st = 0; st < 4; ++st) v += __int_as_float(dpp_row_step(__float_as_int(v), st));
  return v;
}
__device__ __forceinline__ double row16_sum(double v) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int lo = dpp_row_step(__double2loint(v), st), hi = dpp_row_step(__double2hiint(v), st);
    v += __hiloint2double(hi, lo);
  }
  return v;
}

// A block of padded size B = 16 m (m = 2..4) in symmetric storage: strip I
// holds row tile I's columns 16 I .. B-1 (the quarters H_IJ, J >= I) as the
// single 16-row tile of a block of padded size B - 16 I. The lane holds its
// fragment of every strip; z_I = sum_{J >= I} H_IJ r_J + sum_{J < I} H_JI^T r_J.
template <int B, int P>
struct SymB {
  static constexpr int M = B / 16;
  static_assert(M >= 2 && M <= 4, "symmetric storage holds blocks of 32 to 64");
  static constexpr int W1 = M >= 2 ? B - 16 : 16, W2 = M >= 3 ? B - 32 : 16, W3 = M >= 4 ? B - 48 : 16;
  Frag<B, P> f0;
  Frag<W1, P> f1;
  Frag<W2, P> f2;
  Frag<W3, P> f3;
  using CT = std::conditional_t<P == P64, double, float>;

  template <bool NT = false>
  __device__ __forceinline__ void load(const uint8_t *blk, int lane) {
    constexpr int BY = prec_bytes(P);
    f0.template load<NT>(blk, 0, lane);
    f1.template load<NT>(blk + (int64_t)sym_strip_off(B, 1) * BY, 0, lane);
    if constexpr (M >= 3) f2.template load<NT>(blk + (int64_t)sym_strip_off(B, 2) * BY, 0, lane);
    if constexpr (M >= 4) f3.template load<NT>(blk + (int64_t)sym_strip_off(B, 3) * BY, 0, lane);
  }

  // lane (i, kq)'s share of (H_JI^T r_J)[4 s + kq] for every J < I: its entry
  // H_JI[i][4 s + kq] is k-step 4 (I - J) + s of strip J's fragment
  template <int I, int S>
  __device__ __forceinline__ CT trans_term(const CT (&ri)[4]) const {
    CT t = f0.template value<4 * I + S>() * ri[0];
    if constexpr (I >= 2) t += f1.template value<4 * (I - 1) + S>() * ri[1];
    if constexpr (I >= 3) t += f2.template value<4 * (I - 2) + S>() * ri[2];
    return t;
  }

  // the transposed contributions to row tile I, summed over the 16 lanes of
  // each column class (one DPP row) and left in tt[16 I + 4 s + kq]
  template <int I>
  __device__ __forceinline__ void trans(const CT (&ri)[4], double *tt, int lane) const {
    const int i = lane & 15, kq = lane >> 4;
    CT t0 = row16_sum(trans_term<I, 0>(ri)), t1 = row16_sum(trans_term<I, 1>(ri));
    CT t2 = row16_sum(trans_term<I, 2>(ri)), t3 = row16_sum(trans_term<I, 3>(ri));
    if (i < 4) tt[16 * I + 4 * i + kq] = (double)(i == 0 ? t0 : i == 1 ? t1 : i == 2 ? t2 : t3);
  }

  // r32 / r64: the block's residual in LDS; writes sc * (H r) to zt[0..B-1];
  // tt: B LDS slots of scratch
  __device__ __forceinline__ void apply(const float *r32, const double *r64, double sc, double *zt, double *tt,
                                        int lane) const {
    const int i = lane & 15;
    double zd[4];
    zd[0] = f0.dot(r32, r64, lane);
    zd[1] = f1.dot(r32 + 16, r64 + 16, lane);
    if constexpr (M >= 3) zd[2] = f2.dot(r32 + 32, r64 + 32, lane);
    if constexpr (M >= 4) zd[3] = f3.dot(r32 + 48, r64 + 48, lane);
    CT ri[4];
#pragma unroll
    for (int J = 0; J < M - 1; ++J) {
      if constexpr (P == P64) ri[J] = r64[16 * J + i];
      else ri[J] = r32[16 * J + i];
    }
    trans<1>(ri, tt, lane);
    if constexpr (M >= 3) trans<2>(ri, tt, lane);
    if constexpr (M >= 4) trans<3>(ri, tt, lane);
    wave_lds_sync();
    if (lane < 16) {
      zt[lane] = zd[0] * sc;
#pragma unroll
      for (int I = 1; I < M; ++I) zt[16 * I + lane] = (zd[I] + tt[16 * I + lane]) * sc;
    }
  }
};

template <int B, int P, bool NT>
__device__ __forceinline__ void sym_apply(const uint8_t *blk, const float *r32, const double *r64, double sc,
                                          double *zt, double *tt, int lane) {
  SymB<B, P> f;
  f.template load<NT>(blk, lane);
  f.apply(r32, r64, sc, zt, tt, lane);
}

template <int B, bool NT>
__device__ __forceinline__ void sym_apply_p(int prec, const uint8_t *blk, const float *r32, const double *r64,
                                            double sc, double *zt, double *tt, int lane) {
  switch (prec) {
    case P64: sym_apply<B, P64, NT>(blk, r32, r64, sc, zt, tt, lane); break;
    case P32: sym_apply<B, P32, NT>(blk, r32, r64, sc, zt, tt, lane); break;
    case PBF16: sym_apply<B, PBF16, NT>(blk, r32, r64, sc, zt, tt, lane); break;
    default: sym_apply<B, P16, NT>(blk, r32, r64, sc, zt, tt, lane); break;
  }
}

__device__ __forceinline__ void record_high(PcgState *st, int idx, int hi) {
  if (st->high_hist && idx >= 0 && idx <= st->maxit) st->high_hist[idx] = (uint8_t)hi;
}

__device__ __forceinline__ bool temporal_high(const PcgState *st, double relres) {
  if (st->temporal == BJAC_TEMPORAL_HL) return relres >= st->adp_tol;
  if (st->temporal == BJAC_TEMPORAL_LH) return !(relres >= st->adp_tol);
  return false;
}

// State transition after the r update (rr known): iteration count, relres,
// convergence, the switch decision for the next application.
__device__ __forceinline__ void after_update(PcgState *st, double rr) {
  st->rr = rr;
  if (st->restart) {
    // r was replaced by b - A x (alpha = 0, no x update): new relres only
    st->relres = sqrt(rr) / st->rnorm0;
  } else if (st->iter < 0) {
    st->rnorm0 = sqrt(rr);
    st->iter = 0;
    st->relres = INFINITY;
    if (st->rnorm0 == 0.0) {
      st->relres = 0.0;
      st->status = ST_CONVERGED;
    }
  } else {
    st->iter += 1;
    st->relres = sqrt(rr) / st->rnorm0;
    if (st->relres_hist) st->relres_hist[st->iter - 1] = st->relres;
    if (st->relres <= st->tol) st->status = ST_CONVERGED;
  }
  st->use_high = temporal_high(st, st->relres) ? 1 : 0;
}

// State transition after the application (rz known).
__device__ __forceinline__ void after_apply(PcgState *st, double rz, int used_high) {
  st->rz = rz;
  record_high(st, st->iter, used_high);
  st->n_high += used_high;
  if (!(rz > 0.0)) {
    st->status = ST_BREAKDOWN;
    return;
  }
  // a restart begins a new direction sequence: p = z
  st->beta = (st->iter == 0 || st->restart) ? 0.0 : rz / st->rho;
  st->rho = rz;
  st->restart = 0;
  if (st->iter >= st->maxit) st->status = ST_MAXIT;
}

template <int MODE>
struct ModeTraits {
  static constexpr bool UPD = MODE == M_FUSED || MODE == M_UPD;
  static constexpr bool CG = MODE == M_CG;
  static constexpr bool APP = MODE != M_UPD;
  static constexpr bool PCG = MODE != M_APP;
};

// Row phase of one lane (x += alpha p, r -= alpha q in the update modes; the
// p / s recurrences first in the single-reduction mode; else read r), split
// into loads and stores: the kernels hold a tile's stores back until the next
// tile's loads are out, because a wait for loads also waits for every store
// issued before them (one counter), so storing at the end of a tile would add
// a store round trip to every tile. Loads read a row clamped into [0, n) and
// are zeroed for lanes without a row, so no branch separates them.
struct RowIn {
  double x, p, q, r, u, w;
};

// Results of one tile, stored after the next tile's loads are issued.
struct RowHold {
  bool real = false;
  int grow = 0;
  double x = 0.0, r = 0.0, z = 0.0, p = 0.0, s = 0.0;
};

struct UpdCoef {
  double alpha, beta;
};

template <int MODE>
__device__ __forceinline__ UpdCoef upd_coef(const ApplyArgs &a) {
  UpdCoef c{0.0, 0.0};
  if constexpr (ModeTraits<MODE>::UPD || ModeTraits<MODE>::CG) c.alpha = a.st->alpha;
  if constexpr (ModeTraits<MODE>::CG) c.beta = a.st->beta;
  return c;
}

template <int MODE, bool NT = false>
__device__ __forceinline__ RowIn row_load(const ApplyArgs &a, bool real, int grow) {
  const int gc = min(max(grow, 0), a.n - 1);
  RowIn v{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if constexpr (ModeTraits<MODE>::UPD) {
    v.x = ld_hint<NT>(a.x + gc);
    v.p = ld_hint<NT>(a.p + gc);
    v.q = ld_hint<NT>(a.q + gc);
    v.r = ld_hint<NT>(a.r + gc);
  } else if constexpr (ModeTraits<MODE>::CG) {
    v.x = ld_hint<NT>(a.x + gc);
    v.p = ld_hint<NT>(a.pw + gc);
    v.q = ld_hint<NT>(a.sw + gc);
    v.r = ld_hint<NT>(a.r + gc);
    v.u = ld_hint<NT>(a.z + gc);
    v.w = ld_hint<NT>(a.q + gc);
  } else if constexpr (MODE == M_APP) {
    v.r = a.rin[gc];
  } else {
    v.r = ld_hint<NT>(a.r + gc);
  }
  if (!real) v = RowIn{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  return v;
}

// The update of one row; returns the residual the application reads and
// leaves the row's new x (and p, s) in h.
template <int MODE>
__device__ __forceinline__ double row_update(const RowIn &v, const UpdCoef &c, double &rr, RowHold &h) {
  if constexpr (ModeTraits<MODE>::UPD) {
    h.x = fma(c.alpha, v.p, v.x);
    const double rv = fma(-c.alpha, v.q, v.r);
    rr = fma(rv, rv, rr);
    return rv;
  } else if constexpr (ModeTraits<MODE>::CG) {
    h.p = fma(c.beta, v.p, v.u);
    h.s = fma(c.beta, v.q, v.w);
    h.x = fma(c.alpha, h.p, v.x);
    return fma(-c.alpha, h.s, v.r);
  } else {
    return v.r;
  }
}

template <int MODE, bool NT = false>
__device__ __forceinline__ void row_store(const ApplyArgs &a, const RowHold &h) {
  if (!h.real) return;
  if constexpr (ModeTraits<MODE>::UPD || ModeTraits<MODE>::CG) {
    st_hint<NT>(h.x, a.x + h.grow);
    st_hint<NT>(h.r, a.r + h.grow);
  }
  if constexpr (ModeTraits<MODE>::CG) {
    st_hint<NT>(h.p, a.pw + h.grow);
    st_hint<NT>(h.s, a.sw + h.grow);
  }
  if constexpr (ModeTraits<MODE>::APP) st_hint<NT>(h.z, a.z + h.grow);
}

// Reductions and the state machine at the end of a PCG launch.
template <int MODE>
__device__ __forceinline__ void apply_epilogue(const ApplyArgs &a, double rr, double rz, double *sh, int *flag) {
  using T = ModeTraits<MODE>;
  if constexpr (T::CG) return;   // the single-reduction SpMV takes the dots
  const double brr = T::UPD ? block_sum(rr, sh) : 0.0;
  const double brz = T::APP ? block_sum(rz, sh) : 0.0;
  if (threadIdx.x == 0) {
    if (T::UPD) publish(a.part + 2 * blockIdx.x, brr);
    if (T::APP) publish(a.part + 2 * blockIdx.x + 1, brz);
    flag[1] = 1;
  }
  uint32_t *ticket = T::UPD ? &a.st->ticket_b : &a.st->ticket_c;
  if (last_workgroup(ticket, flag)) {
    double trr = 0.0, trz = 0.0;
    if constexpr (T::UPD && T::APP) {
      double both[2];
      sum_partials_n<2>(a.part, gridDim.x, 2, sh, flag + 1, both);
      trr = both[0];
      trz = both[1];
    } else if constexpr (T::UPD) {
      trr = sum_partials(a.part, gridDim.x, 2, sh, flag + 1);
    } else {
      trz = sum_partials(a.part + 1, gridDim.x, 2, sh, flag + 1);
    }
    if (threadIdx.x == 0) {
      PcgState *st = a.st;
      if (!flag[1]) {
        st->status = ST_SYNC_FAIL;
      } else {
        if (T::UPD) after_update(st, trr);
        if (T::APP && st->status == ST_RUNNING) after_apply(st, trz, MODE == M_APPDEV ? a.want_high : 0);
      }
      __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Launches whose map does not match the device-side switch exit at once.
template <int MODE>
__device__ __forceinline__ bool apply_skip(const ApplyArgs &a) {
  if (ModeTraits<MODE>::PCG && a.st->status != ST_RUNNING) return true;
  if (MODE == M_APPDEV && ((a.st->use_high != 0) != (a.want_high != 0))) return true;
  return false;
}

// Fast path: every block but the last has B rows, the map stores every block
// in P, block k at a fixed stride. Rows, block addresses and the tile shape are
// arithmetic, so the stored fragments, the per-block scales and the vectors of
// a tile are all requested before the first wait.
// SYM: blocks of 32 to 64 in symmetric storage (the quarters below the
// diagonal taken as transposes of stored ones).
template <int B, int P, int MODE, bool SYM = false, bool NT = false>
__global__ __launch_bounds__(256) void apply_fast_kernel(ApplyArgs a) {
  static_assert(!SYM || B >= 32, "symmetric storage holds blocks of 32 to 64");
  using T = ModeTraits<MODE>;
  constexpr int NB = 64 / B;        // blocks per wave tile
  constexpr int R = NB * B;         // padded rows per wave tile
  constexpr int MT = R / 16;        // 16-row tiles per wave tile
  constexpr int MPB = B / 16;       // 16-row tiles per block
  using F = Frag<B, P>;
  constexpr int64_t BLK = (SYM ? (int64_t)sym_elems(B) : (int64_t)B * B) * prec_bytes(P);
  constexpr bool PRE = SYM || MT * F::G <= 8;
  __shared__ float r32s[4][64];
  __shared__ double r64s[4][64];
  __shared__ double zts[4][64];
  __shared__ double tts[4][SYM ? 64 : 1];
  __shared__ double sh[4];
  __shared__ int flag[2];
  if (apply_skip<MODE>(a)) return;
  const UpdCoef cf = upd_coef<MODE>(a);
  const uint8_t *__restrict__ base = a.map.base + a.off0;
  const double *__restrict__ scale = a.map.scale;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float *r32 = r32s[wv];
  double *r64 = r64s[wv];
  double *zt = zts[wv];
  const int j = lane / B, li = lane - j * B;
  double rr = 0.0, rz = 0.0;
  RowHold hold;   // results of the previous tile, stored after this tile's loads
  for (WaveIter it(a.ntiles); it.t < it.end; it.t += it.step) {
    const int k0 = it.t * NB;
    const int kb = k0 + j;
    const int grow = kb * B + li;
    const bool real = lane < R && kb < a.nb && grow < a.n;
    F fr[PRE && !SYM ? MT : 1];
    SymB<SYM ? B : 32, P> fs[SYM ? NB : 1];
    double scl = 1.0;
    if constexpr (T::APP) {
      if constexpr (P != P64) scl = scale[min(k0 + lane % NB, a.nb - 1)];
      if constexpr (SYM) {
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) fs[jb].template load<NT>(base + (int64_t)min(k0 + jb, a.nb - 1) * BLK, lane);
      } else if constexpr (PRE) {
#pragma unroll
        for (int u = 0; u < MT; ++u)
          fr[u].template load<NT>(base + (int64_t)min(k0 + u / MPB, a.nb - 1) * BLK, u % MPB, lane);
      }
    }
    const RowIn v = row_load<MODE, NT>(a, real, grow);
    row_store<MODE, NT>(a, hold);
    RowHold nh;
    const double rv = row_update<MODE>(v, cf, rr, nh);
    double zv_out = 0.0;
    if constexpr (T::APP) {
      if (lane < R) {
        r64[lane] = rv;
        r32[lane] = __double2float_rn(rv);
      }
      wave_lds_sync();
      if constexpr (SYM) {
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
          if (k0 + jb < a.nb) {
            const int cb = jb * B;
            const double sc = (P == P64) ? 1.0 : bcast(scl, jb);
            fs[jb].apply(r32 + cb, r64 + cb, sc, zt + cb, tts[wv] + cb, lane);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < (SYM ? 0 : MT); ++u) {
        const int jb = u / MPB;
        if (k0 + jb < a.nb) {
          const int cb = jb * B;
          double zv;
          if constexpr (PRE) {
            zv = fr[u].dot(r32 + cb, r64 + cb, lane);
          } else {
            F f;
            f.template load<NT>(base + (int64_t)(k0 + jb) * BLK, u % MPB, lane);
            zv = f.dot(r32 + cb, r64 + cb, lane);
          }
          const double sc = (P == P64) ? 1.0 : bcast(scl, jb);
          if (lane < 16) zt[cb + (u % MPB) * 16 + lane] = zv * sc;
        }
      }
      wave_lds_sync();
      if (real) {
        zv_out = zt[lane];
        rz = fma(rv, zv_out, rz);
      }
    }
    nh.real = real;
    nh.grow = grow;
    nh.r = rv;
    nh.z = zv_out;
    hold = nh;
  }
  row_store<MODE, NT>(a, hold);
  if (T::PCG) apply_epilogue<MODE>(a, rr, rz, sh, flag);
}

template <int B, bool NT>
__device__ __forceinline__ double mtile_dot(int prec, const uint8_t *blk, int mt, const float *r32, const double *r64,
                                            int lane) {
  switch (prec) {
    case P64: { Frag<B, P64> f; f.template load<NT>(blk, mt, lane); return f.dot(r32, r64, lane); }
    case P32: { Frag<B, P32> f; f.template load<NT>(blk, mt, lane); return f.dot(r32, r64, lane); }
    case PBF16: { Frag<B, PBF16> f; f.template load<NT>(blk, mt, lane); return f.dot(r32, r64, lane); }
    default: { Frag<B, P16> f; f.template load<NT>(blk, mt, lane); return f.dot(r32, r64, lane); }
  }
}

__device__ __forceinline__ int readlane_i(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ int64_t readlane_l(int64_t v, int src) {
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), src);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), src);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Generic path: blocks of different sizes and/or precisions. Each wave tile
// (up to 4 blocks, at most 64 padded rows, from the setup's tile list) reads
// its blocks' metadata with one lane-parallel load per array and broadcasts it;
// each 16-row tile dispatches on its block's size and precision.
template <int MODE, bool NT = false>
__global__ __launch_bounds__(256) void apply_generic_kernel(ApplyArgs a) {
  using T = ModeTraits<MODE>;
  __shared__ float r32s[4][64];
  __shared__ double r64s[4][64];
  __shared__ double zts[4][64];
  __shared__ double tts[4][64];
  __shared__ double sh[4];
  __shared__ int flag[2];
  if (apply_skip<MODE>(a)) return;
  const UpdCoef cf = upd_coef<MODE>(a);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float *r32 = r32s[wv];
  double *r64 = r64s[wv];
  double *zt = zts[wv];
  double rr = 0.0, rz = 0.0;
  RowHold hold;   // results of the previous tile, stored after this tile's loads
  for (WaveIter it(a.ntiles); it.t < it.end; it.t += it.step) {
    const int k0 = __builtin_amdgcn_readfirstlane(a.tile_blk[it.t]);
    const int nk = __builtin_amdgcn_readfirstlane(a.tile_blk[it.t + 1]) - k0;
    const int kl = k0 + min(lane, nk - 1);
    const int mB = a.bpad[kl], mrow = a.blk_row[kl], mrow1 = a.blk_row[kl + 1];
    int64_t moff = 0;
    double msc = 1.0;
    int mtag = 0;
    if constexpr (T::APP) {
      moff = a.map.off[kl];
      msc = a.map.scale[kl];
      mtag = a.map.tag[kl];
    }
    int cum = 0, row0 = 0, bsz = 0, li = -1;
    for (int i = 0; i < nk; ++i) {
      const int Bi = readlane_i(mB, i);
      if (lane >= cum && lane < cum + Bi) {
        li = lane - cum;
        row0 = readlane_i(mrow, i);
        bsz = readlane_i(mrow1, i) - row0;
      }
      cum += Bi;
    }
    const bool real = li >= 0 && li < bsz;
    const int grow = row0 + li;
    const RowIn v = row_load<MODE, NT>(a, real, grow);
    row_store<MODE, NT>(a, hold);
    RowHold nh;
    const double rv = row_update<MODE>(v, cf, rr, nh);
    double zv_out = 0.0;
    if constexpr (T::APP) {
      if (lane < cum) {
        r64[lane] = rv;
        r32[lane] = __double2float_rn(rv);
      }
      wave_lds_sync();
      int cb = 0;
      for (int i = 0; i < nk; ++i) {
        const int B = readlane_i(mB, i);
        const int prec = readlane_i(mtag, i);
        const uint8_t *blk = a.map.base + readlane_l(moff, i);
        const double sc = bcast(msc, i);
        if (B >= 32 && a.map.sym) {
          switch (B) {
            case 32: sym_apply_p<32, NT>(prec, blk, r32 + cb, r64 + cb, sc, zt + cb, tts[wv] + cb, lane); break;
            case 48: sym_apply_p<48, NT>(prec, blk, r32 + cb, r64 + cb, sc, zt + cb, tts[wv] + cb, lane); break;
            default: sym_apply_p<64, NT>(prec, blk, r32 + cb, r64 + cb, sc, zt + cb, tts[wv] + cb, lane); break;
          }
          cb += B;
          continue;
        }
        for (int mt = 0; mt < B / 16; ++mt) {
          double zv;
          switch (B) {
            case 16: zv = mtile_dot<16, NT>(prec, blk, mt, r32 + cb, r64 + cb, lane); break;
            case 32: zv = mtile_dot<32, NT>(prec, blk, mt, r32 + cb, r64 + cb, lane); break;
            case 48: zv = mtile_dot<48, NT>(prec, blk, mt, r32 + cb, r64 + cb, lane); break;
            default: zv = mtile_dot<64, NT>(prec, blk, mt, r32 + cb, r64 + cb, lane); break;
          }
          if (lane < 16) zt[cb + mt * 16 + lane] = zv * sc;
        }
        cb += B;
      }
      wave_lds_sync();
      if (real) {
        zv_out = zt[lane];
        rz = fma(rv, zv_out, rz);
      }
    }
    nh.real = real;
    nh.grow = grow;
    nh.r = rv;
    nh.z = zv_out;
    hold = nh;
  }
  row_store<MODE, NT>(a, hold);
  if (T::PCG) apply_epilogue<MODE>(a, rr, rz, sh, flag);
}

// Band-stored maps: block k keeps the diagonals d = 0..w_k of its symmetric
// inverse, diagonal d as bpad_k entries E(d, j) = H[j][j + d] (zero where
// j + d >= b_k) at base + off[k] + (d * bpad_k + j) * bytes. Lane li of a
// block forms
//   z_li = s_k (sum_{d=0}^{w_k} E(d, li) r_{li+d} + sum_{d=1}^{w_k} E(d, li-d) r_{li-d})
// and loads only its own E(d, li): E(d, li - d) and r_{li+-d} are the values
// of lanes li -+ d, moved across the wave. The blocks of a wave tile sit on
// consecutive lanes, so lane li - d belongs to the same block exactly when
// li >= d, and E(d, li) = 0 wherever li + d leaves the block. Diagonals are
// loaded eight at a time, all in flight before the first product; the lane
// moves run in wave-uniform control flow.
__device__ __forceinline__ double fma_t(double x, double y, double z) { return fma(x, y, z); }
__device__ __forceinline__ float fma_t(float x, float y, float z) { return fmaf(x, y, z); }

// The band product of one lane: li is the lane's row in its block (-1: no
// block), Bp the block's padded size, wl its half-bandwidth, wmax the largest
// half-bandwidth of the wave (wave-uniform), tg its precision, sc its scale.
// PU: the precision of every block of the map, or -1 (per-block tags; FP64
// blocks in FP64, the others in FP32 on the FP32 copy of r).
// Eight diagonals are taken per round, with no branch inside a round: the
// loads read positions clamped into the lane's own block (d -> min(d, w),
// li -> max(li, 0)), so all eight are in flight together, and entries past
// the lane's width are zeroed (a branch would let the compiler sink loads
// behind it and wait for each in turn). The lane moves go four at a time.
// A mixed map loads the 8-byte-aligned word holding each entry (every block
// starts on a 32-byte boundary and spans a multiple of 32 bytes, so the word
// lies in the block) and picks the entry out of it by format.
constexpr int kBandRound = 8;

template <int PU>
struct BandRaw {
  using T = std::conditional_t<PU == P64, uint64_t,
                               std::conditional_t<PU == P32, uint32_t, std::conditional_t<PU >= 0, uint16_t, uint2>>>;
  T v[kBandRound];
};

template <int PU>
__device__ __forceinline__ void band_load_round(BandRaw<PU> &raw, const uint8_t *__restrict__ blk, int Bp, int lc,
                                                int wc, int d0, int tg) {
  using RT = typename BandRaw<PU>::T;
  if constexpr (PU >= 0) {
    constexpr int BY = prec_bytes(PU);
#pragma unroll
    for (int u = 0; u < kBandRound; ++u) raw.v[u] = *(const RT *)(blk + ((int64_t)min(d0 + u, wc) * Bp + lc) * BY);
  } else {
    const int BY = prec_bytes(tg);
#pragma unroll
    for (int u = 0; u < kBandRound; ++u) {
      const int64_t bo = ((int64_t)min(d0 + u, wc) * Bp + lc) * BY;
      raw.v[u] = *(const uint2 *)(blk + (bo & ~(int64_t)7));
    }
  }
}

// raw0: the first round (diagonals 0..7), already loaded by the caller.
template <int PU>
__device__ __forceinline__ double band_product(const uint8_t *__restrict__ blk, int Bp, int li, int wl, int wmax,
                                               int tg, double sc, double rv, const BandRaw<PU> &raw0) {
  constexpr int DC = kBandRound, DQ = 4;
  const int wc = max(wl, 0), lc = max(li, 0);
  if constexpr (PU >= 0) {
    using CT = std::conditional_t<PU == P64, double, float>;
    CT rc;
    if constexpr (PU == P64) rc = rv;
    else rc = __double2float_rn(rv);
    CT acc = CT(0);
    for (int d0 = 0; d0 <= wmax; d0 += DC) {
      BandRaw<PU> rn;
      if (d0 > 0) band_load_round<PU>(rn, blk, Bp, lc, wc, d0, tg);
      const BandRaw<PU> &raw = d0 > 0 ? rn : raw0;
      CT e[DC];
#pragma unroll
      for (int u = 0; u < DC; ++u) {
        CT v;
        if constexpr (PU == P64) v = __longlong_as_double((long long)raw.v[u]);
        else if constexpr (PU == P32) v = __uint_as_float(raw.v[u]);
        else if constexpr (PU == PBF16) v = __uint_as_float((uint32_t)raw.v[u] << 16);
        else v = f16_bits(raw.v[u]);
        e[u] = (li >= 0 && d0 + u <= wl) ? v : CT(0);
      }
#pragma unroll
      for (int g = 0; g < DC; g += DQ) {
        CT rup[DQ], rdn[DQ], elo[DQ];
#pragma unroll
        for (int q = 0; q < DQ; ++q) {
          const int d = d0 + g + q;
          rup[q] = __shfl_down(rc, d, kWave);
          rdn[q] = __shfl_up(rc, d, kWave);
          elo[q] = __shfl_up(e[g + q], d, kWave);
        }
#pragma unroll
        for (int q = 0; q < DQ; ++q) {
          const int d = d0 + g + q;
          acc = fma_t(e[g + q], rup[q], acc);
          if (d >= 1 && li >= d) acc = fma_t(elo[q], rdn[q], acc);
        }
      }
    }
    return (PU == P64) ? (double)acc : (double)acc * sc;
  } else {
    const bool f64 = tg == P64;
    const int BY = prec_bytes(tg);
    const float r32 = __double2float_rn(rv);
    double acc64 = 0.0;
    float acc32 = 0.0f;
    for (int d0 = 0; d0 <= wmax; d0 += DC) {
      BandRaw<PU> rn;
      if (d0 > 0) band_load_round<PU>(rn, blk, Bp, lc, wc, d0, tg);
      const BandRaw<PU> &raw = d0 > 0 ? rn : raw0;
      double e[DC];
#pragma unroll
      for (int u = 0; u < DC; ++u) {
        const int b4 = (int)((((int64_t)min(d0 + u, wc) * Bp + lc) * BY) & 7);
        const uint32_t w32 = (b4 & 4) ? raw.v[u].y : raw.v[u].x;
        const uint32_t h16 = (b4 & 2) ? (w32 >> 16) : (w32 & 0xffffu);
        double v;
        if (tg == P64) v = __hiloint2double((int)raw.v[u].y, (int)raw.v[u].x);
        else if (tg == P32) v = (double)__uint_as_float(w32);
        else if (tg == PBF16) v = (double)__uint_as_float(h16 << 16);
        else v = (double)f16_bits((uint16_t)h16);
        e[u] = (li >= 0 && d0 + u <= wl) ? v : 0.0;
      }
#pragma unroll
      for (int g = 0; g < DC; g += DQ) {
        double rup[DQ], rdn[DQ], elo[DQ];
#pragma unroll
        for (int q = 0; q < DQ; ++q) {
          const int d = d0 + g + q;
          rup[q] = __shfl_down(rv, d, kWave);
          rdn[q] = __shfl_up(rv, d, kWave);
          elo[q] = __shfl_up(e[g + q], d, kWave);
        }
#pragma unroll
        for (int q = 0; q < DQ; ++q) {
          const int d = d0 + g + q;
          const bool lower = d >= 1 && li >= d;
          if (f64) {
            acc64 = fma(e[g + q], rup[q], acc64);
            if (lower) acc64 = fma(elo[q], rdn[q], acc64);
          } else {
            acc32 = fmaf((float)e[g + q], __double2float_rn(rup[q]), acc32);
            if (lower) acc32 = fmaf((float)elo[q], __double2float_rn(rdn[q]), acc32);
          }
        }
      }
    }
    return f64 ? acc64 : (double)acc32 * sc;
  }
}

// Generic band path: blocks of different sizes; the wave tiles of the setup.
template <int MODE, int PU>
__global__ __launch_bounds__(256) void apply_band_kernel(ApplyArgs a) {
  using T = ModeTraits<MODE>;
  __shared__ double sh[4];
  __shared__ int flag[2];
  if (apply_skip<MODE>(a)) return;
  const UpdCoef cf = upd_coef<MODE>(a);
  const int lane = threadIdx.x & 63;
  double rr = 0.0, rz = 0.0;
  RowHold hold;   // results of the previous tile, stored after this tile's loads
  for (WaveIter it(a.ntiles); it.t < it.end; it.t += it.step) {
    const int k0 = __builtin_amdgcn_readfirstlane(a.tile_blk[it.t]);
    const int nk = __builtin_amdgcn_readfirstlane(a.tile_blk[it.t + 1]) - k0;
    const int kl = k0 + min(lane, nk - 1);
    const int mB = a.bpad[kl], mrow = a.blk_row[kl], mrow1 = a.blk_row[kl + 1];
    const int64_t moff = a.map.off[kl];
    const double msc = a.map.scale[kl];
    const int mtag = a.map.tag[kl], mw = a.map.w[kl];
    int cum = 0, row0 = 0, bsz = 0, li = -1, Bp = 0, wl = -1, tg = 0, wmax = 0;
    int64_t off = 0;
    double sc = 1.0;
    for (int i = 0; i < nk; ++i) {
      const int Bi = readlane_i(mB, i);
      const int wi = readlane_i(mw, i);
      const int64_t oi = readlane_l(moff, i);
      const double si = bcast(msc, i);
      const int ti = readlane_i(mtag, i);
      const int r0i = readlane_i(mrow, i);
      const int r1i = readlane_i(mrow1, i);
      wmax = max(wmax, wi);
      if (lane >= cum && lane < cum + Bi) {
        li = lane - cum;
        row0 = r0i;
        bsz = r1i - r0i;
        Bp = Bi;
        wl = wi;
        off = oi;
        sc = si;
        tg = ti;
      }
      cum += Bi;
    }
    const bool real = li >= 0 && li < bsz;
    const int grow = row0 + li;
    BandRaw<PU> raw0;
    band_load_round<PU>(raw0, a.map.base + off, Bp, max(li, 0), max(wl, 0), 0, tg);
    const RowIn v = row_load<MODE>(a, real, grow);
    row_store<MODE>(a, hold);
    RowHold nh;
    const double rv = row_update<MODE>(v, cf, rr, nh);
    const double zv = band_product<PU>(a.map.base + off, Bp, li, wl, wmax, tg, sc, rv, raw0);
    if (real) rz = fma(rv, zv, rz);
    nh.real = real;
    nh.grow = grow;
    nh.r = rv;
    nh.z = zv;
    hold = nh;
  }
  row_store<MODE>(a, hold);
  if (T::PCG) apply_epilogue<MODE>(a, rr, rz, sh, flag);
}

// Fast band path: every block but the last has B rows (B = 16, 32, 48, 64),
// so rows and blocks of a wave tile are arithmetic. Each lane fetches the
// offset and width of its block in the wave's next tile one tile ahead, so the
// diagonal loads of a tile go out together with its vector loads.
template <int B, int MODE, int PU>
__global__ __launch_bounds__(256) void apply_band_fast_kernel(ApplyArgs a) {
  using T = ModeTraits<MODE>;
  constexpr int NB = 64 / B;
  constexpr int R = NB * B;
  __shared__ double sh[4];
  __shared__ int flag[2];
  if (apply_skip<MODE>(a)) return;
  const UpdCoef cf = upd_coef<MODE>(a);
  const int lane = threadIdx.x & 63;
  const int j = lane / B, li0 = lane - j * B;
  double rr = 0.0, rz = 0.0;
  WaveIter it(a.ntiles);
  // block indices are clamped to the last block, so every fetch is in bounds
  int kn = min(it.t * NB + j, a.nb - 1);
  int64_t off_n = a.map.off[kn];
  int w_n = a.map.w[kn];
  RowHold hold;   // results of the previous tile, stored after this tile's loads
  for (; it.t < it.end; it.t += it.step) {
    const int kb = it.t * NB + j;
    const int kc = min(kb, a.nb - 1);
    const int grow = kb * B + li0;
    const bool inb = lane < R && kb < a.nb;
    const bool real = inb && grow < a.n;
    const int64_t off = off_n;
    const int wl = inb ? w_n : -1;
    kn = min((it.t + it.step) * NB + j, a.nb - 1);
    off_n = a.map.off[kn];
    w_n = a.map.w[kn];
    const double sc = PU == P64 ? 1.0 : a.map.scale[kc];
    const int tg = PU >= 0 ? PU : (int)a.map.tag[kc];
    BandRaw<PU> raw0;
    band_load_round<PU>(raw0, a.map.base + off, B, inb ? li0 : 0, max(wl, 0), 0, tg);
    const RowIn v = row_load<MODE>(a, real, grow);
    row_store<MODE>(a, hold);   // the previous tile's results
    RowHold nh;
    const double rv = row_update<MODE>(v, cf, rr, nh);
    int wmax = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) wmax = max(wmax, readlane_i(wl, q * B));
    const double zv = band_product<PU>(a.map.base + off, B, inb ? li0 : -1, wl, wmax, tg, sc, rv, raw0);
    if (real) rz = fma(rv, zv, rz);
    nh.real = real;
    nh.grow = grow;
    nh.r = rv;
    nh.z = zv;
    hold = nh;
  }
  row_store<MODE>(a, hold);
  if (T::PCG) apply_epilogue<MODE>(a, rr, rz, sh, flag);
}

// ------------------------------------------------------------ small kernels
__global__ void state_init_kernel(PcgState *st, double tol, int maxit, double adp_tol, int temporal,
                                  double *relres_hist, uint8_t *high_hist) {
  PcgState s{};
  s.cidx = 1;   // the index compaction kernels lower or raise it
  s.tol = tol;
  s.maxit = maxit;
  s.adp_tol = adp_tol;
  s.temporal = temporal;
  s.iter = -1;
  s.status = ST_RUNNING;
  s.alpha = 0.0;
  s.relres = INFINITY;
  s.relres_hist = relres_hist;
  s.high_hist = high_hist;
  // the first application sees relres = +inf: hl starts high, lh starts low
  s.use_high = temporal == BJAC_TEMPORAL_HL ? 1 : 0;
  *st = s;
}

// x = 0, r = b and zeros in the work vectors the first iteration reads (the
// single-reduction form also reads u and s, scaled by beta = 0)
__global__ __launch_bounds__(256) void pcg_fill_kernel(int64_t n, double *x, double *r, const double *b, double *p,
                                                       double *q, double *u, double *s) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    x[i] = 0.0;
    r[i] = b[i];
    p[i] = 0.0;
    q[i] = 0.0;
    if (u) u[i] = 0.0;
    if (s) s[i] = 0.0;
  }
}

// r = b - A x in FP64 with per-workgroup partial sums of r^2 (true-residual
// verification; one thread per row, grid-stride).
__global__ __launch_bounds__(256) void resid_kernel(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                                                    const double *x, const double *b, double *r, double *part) {
  __shared__ double sh[4];
  double acc2 = 0.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double ax = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) ax = fma(v[k], x[ci[k]], ax);
    const double ri = b[i] - ax;
    r[i] = ri;
    acc2 = fma(ri, ri, acc2);
  }
  const double t = block_sum(acc2, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Sums the partials in order; if ||b - A x|| / ||b|| > tol, CG continues from
// the replaced residual: the next application runs with alpha = 0 and starts
// a new direction sequence.
__global__ __launch_bounds__(256) void restart_kernel(PcgState *st, const double *part, int G) {
  __shared__ double sh[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < G; i += 256) v += part[i];
  const double rr = block_sum(v, sh);
  if (threadIdx.x == 0) {
    st->rr_true = rr;
    if (st->status == ST_CONVERGED && sqrt(rr) > st->tol * st->rnorm0 && st->iter < st->maxit) {
      st->status = ST_RUNNING;
      st->alpha = 0.0;
      st->beta = 0.0;
      st->restart = 1;
    }
  }
}

__global__ __launch_bounds__(256) void round_kernel(const double *in, uint8_t *out, int64_t count, int prec,
                                                    double inv_scale) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
    const double v = in[i] * inv_scale;
    if (prec == P32) ((uint32_t *)out)[i] = to_f32_bits(v);
    else if (prec == PBF16) ((uint16_t *)out)[i] = (uint16_t)to_bf16_bits(v);
    else ((uint16_t *)out)[i] = (uint16_t)to_f16_bits(v);
  }
}

int launch_round(const double *in, void *out, int64_t count, int prec, double scale, hipStream_t s) {
  if (count <= 0) return BJAC_OK;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(round_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, (uint8_t *)out, count, prec,
                     1.0 / scale);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}

// ------------------------------------------------ paper-mode BJAC(k, t)
// Eq. 3-1 with k outer steps z_{j+1} = z_j + Dhat^-1 (r - A z_j), z_1 =
// Dhat^-1 r, where Dhat^-1 is eq. 3-3: t point-Jacobi sweeps y <- y + D^-1 (v -
// D_b y) from y = 0 inside every diagonal block. Every operation runs in T:
// FP32 for the low map (Sec. 3.2: all floating-point work of M^-1(p_l) in p_l,
// r converted on entry, z widened on exit, Algorithm 3.1), FP64 for the high
// map. One thread per row, grid-stride.
struct PolyArgs {
  int64_t n;
  const int32_t *rp, *ci;
  const void *val;           // T values of A
  const void *dinv;          // T reciprocals of the diagonal
  const int32_t *rlo, *rhi;  // column range of each row's block
  PcgState *st;              // null outside PCG
  int want_high;             // temporal handles: launch serves the FP64 (1) or low (0) map
  int temporal;
};

__device__ __forceinline__ bool poly_skip(const PolyArgs &a) {
  if (!a.st) return false;
  if (a.st->status != ST_RUNNING) return true;
  return a.temporal && ((a.st->use_high != 0) != (a.want_high != 0));
}

// v = T(r); y = D^-1 v (the first sweep from y = 0)
template <class T>
__global__ __launch_bounds__(256) void poly_first_kernel(PolyArgs a, const double *r, T *v, T *y) {
  if (poly_skip(a)) return;
  const T *dinv = (const T *)a.dinv;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256) {
    const T vi = (T)r[i];
    v[i] = vi;
    y[i] = dinv[i] * vi;
  }
}

// The two CSR passes of an application, over wave tiles of 64 rows whose CSR
// entries are staged in LDS with coalesced (non-temporal) loads, as in the PCG
// SpMV; each lane then gathers its row's neighbours eight at a time with every
// load in flight (index-clamped, masked entries multiplied by zero):
//   PO_SWEEP: yout = yin + D^-1 (v - D_b yin) [+ add], D_b keeping the entries
//             whose column lies in the row's block;
//   PO_RESID: w = v - A z; y = D^-1 w; with zout (t = 1) zout = z + y.
// Entries are summed in row order.
enum PolyOp { PO_SWEEP = 0, PO_RESID = 1 };

template <class T, int OP>
__device__ __forceinline__ T poly_row_dot(const T *__restrict__ xin, const int *__restrict__ cidx,
                                          const T *__restrict__ vals, int base, int len, int lo, int hi) {
  constexpr int U = 8;
  T acc = T(0);
  for (int k0 = 0; k0 < len; k0 += U) {
    int cs[U];
    T vs[U], g[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int idx = base + min(k0 + k, len - 1);
      cs[k] = cidx[idx];
      const T vv = vals[idx];
      const bool keep = k0 + k < len && (OP == PO_RESID || (cs[k] >= lo && cs[k] < hi));
      vs[k] = keep ? vv : T(0);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) g[k] = xin[cs[k]];
#pragma unroll
    for (int k = 0; k < U; ++k) acc = fma_t(vs[k], g[k], acc);
  }
  return acc;
}

template <class T, int OP>
__global__ __launch_bounds__(256) void poly_csr_kernel(PolyArgs a, const T *v, const T *xin, T *o1, T *o2, T *o3,
                                                       const T *add) {
  constexpr int CAP = kSpmvNnzCap;
  constexpr int NL = CAP / 64;
  __shared__ T svs[4][CAP];
  __shared__ int scs[4][CAP];
  if (poly_skip(a)) return;
  const T *__restrict__ val = (const T *)a.val;
  const T *__restrict__ dinv = (const T *)a.dinv;
  const int32_t *__restrict__ rp = a.rp;
  const int32_t *__restrict__ ci = a.ci;
  const int n = (int)a.n;
  const int ntiles = (n + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T *sv = svs[wv];
  int *sc = scs[wv];
  for (WaveIter it(ntiles); it.t < it.end; it.t += it.step) {
    const int r0 = it.t * 64;
    const int r1 = min(n, r0 + 64);
    const int row = r0 + lane;
    const bool has = row < r1;
    const int rowc = min(row, r1 - 1);
    const int s = rp[rowc], e = rp[rowc + 1];
    const int e0 = __builtin_amdgcn_readlane(s, 0);
    const int cnt = __builtin_amdgcn_readlane(e, r1 - 1 - r0) - e0;
    const int len = has ? e - s : 0;
    const int lo = OP == PO_SWEEP ? a.rlo[rowc] : 0;
    const int hi = OP == PO_SWEEP ? a.rhi[rowc] : 0;
    T acc;
    if (cnt > 0 && cnt <= CAP) {
      T vv[NL];
      int cc[NL];
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        const int i = min(lane + 64 * k, cnt - 1);
        vv[k] = __builtin_nontemporal_load(val + e0 + i);
        cc[k] = __builtin_nontemporal_load(ci + e0 + i);
      }
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        const int i = lane + 64 * k;
        if (i < cnt) {
          sv[i] = vv[k];
          sc[i] = cc[k];
        }
      }
      wave_lds_sync();
      acc = poly_row_dot<T, OP>(xin, sc, sv, s - e0, len, lo, hi);
      wave_lds_sync();
    } else {
      acc = poly_row_dot<T, OP>(xin, ci, val, s, len, lo, hi);
    }
    if (has) {
      if constexpr (OP == PO_SWEEP) {
        T yi = xin[row] + dinv[row] * (v[row] - acc);
        if (add) yi = add[row] + yi;
        o1[row] = yi;
      } else {
        const T wi = v[row] - acc;
        o1[row] = wi;
        const T yi = dinv[row] * wi;
        o2[row] = yi;
        if (o3) o3[row] = xin[row] + yi;
      }
    }
  }
}

// z = FP64(zt); in PCG also (r, z) and the state transition after it
template <class T>
__global__ __launch_bounds__(256) void poly_finish_kernel(PolyArgs a, const T *zt, double *z, const double *r,
                                                          double *part) {
  __shared__ double sh[4];
  __shared__ int flag[2];
  if (poly_skip(a)) return;
  double rz = 0.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256) {
    const double zi = (double)zt[i];
    z[i] = zi;
    if (a.st) rz = fma(r[i], zi, rz);
  }
  if (!a.st) return;
  const double brz = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    publish(part + 2 * blockIdx.x + 1, brz);
    flag[1] = 1;
  }
  if (last_workgroup(&a.st->ticket_c, flag)) {
    const double trz = sum_partials(part + 1, gridDim.x, 2, sh, flag + 1);
    if (threadIdx.x == 0) {
      PcgState *st = a.st;
      if (!flag[1]) st->status = ST_SYNC_FAIL;
      else if (st->status == ST_RUNNING) after_apply(st, trz, a.temporal ? a.want_high : 0);
      __hip_atomic_store(&st->ticket_c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

static int poly_grid(int64_t n) { return (int)std::min<int64_t>(kMaxGrid, std::max<int64_t>(1, (n + 255) / 256)); }

// One application z = M^-1 r of a paper-mode handle in precision T.
template <class T>
static void enqueue_poly_app(const bjac_handle *M, PolyArgs a, const double *r, double *z, double *part,
                             hipStream_t s) {
  const int64_t n = M->n;
  const int G = poly_grid(n);
  const int ntiles = (int)((n + 63) / 64);
  const int GC = grid_for_waves(ntiles, (const void *)poly_csr_kernel<T, PO_SWEEP>, kGridPerCuGeneric);
  const int GR = grid_for_waves(ntiles, (const void *)poly_csr_kernel<T, PO_RESID>, kGridPerCuGeneric);
  a.val = sizeof(T) == 4 ? (const void *)M->val32 : (const void *)M->pval;
  a.dinv = sizeof(T) == 4 ? (const void *)M->dinv32 : (const void *)M->dinv64;
  T *v = (T *)M->pbuf, *w = (T *)(M->pbuf + n), *ya = (T *)(M->pbuf + 2 * n), *yb = (T *)(M->pbuf + 3 * n);
  T *za = (T *)(M->pbuf + 4 * n), *zb = (T *)(M->pbuf + 5 * n);
  const int t = M->pt, k = M->pk;
  // block solve of the first outer step, ending in za
  hipLaunchKernelGGL(poly_first_kernel<T>, dim3(G), dim3(256), 0, s, a, r, v, t == 1 ? za : ya);
  {
    T *in = ya, *spare = yb;
    for (int sw = 2; sw <= t; ++sw) {
      T *out = sw == t ? za : spare;
      hipLaunchKernelGGL((poly_csr_kernel<T, PO_SWEEP>), dim3(GC), dim3(256), 0, s, a, (const T *)v, (const T *)in,
                         out, (T *)nullptr, (T *)nullptr, (const T *)nullptr);
      spare = in;
      in = out;
    }
  }
  T *zc = za;
  for (int j = 2; j <= k; ++j) {
    T *zn = zc == za ? zb : za;
    hipLaunchKernelGGL((poly_csr_kernel<T, PO_RESID>), dim3(GR), dim3(256), 0, s, a, (const T *)v, (const T *)zc,
                       w, ya, t == 1 ? zn : (T *)nullptr, (const T *)nullptr);
    T *in = ya, *spare = yb;
    for (int sw = 2; sw <= t; ++sw) {
      T *out = sw == t ? zn : spare;
      hipLaunchKernelGGL((poly_csr_kernel<T, PO_SWEEP>), dim3(GC), dim3(256), 0, s, a, (const T *)w, (const T *)in,
                         out, (T *)nullptr, (T *)nullptr, sw == t ? (const T *)zc : (const T *)nullptr);
      spare = in;
      in = out;
    }
    zc = zn;
  }
  hipLaunchKernelGGL(poly_finish_kernel<T>, dim3(G), dim3(256), 0, s, a, (const T *)zc, z, r, part);
}

static PolyArgs poly_args(const bjac_handle *M, PcgState *st, int want_high) {
  PolyArgs a{};
  a.n = M->n;
  a.rp = M->prp;
  a.ci = M->pci;
  a.rlo = M->rlo;
  a.rhi = M->rhi;
  a.st = st;
  a.want_high = want_high;
  a.temporal = M->policy.temporal != BJAC_TEMPORAL_NONE;
  return a;
}

// the map of a paper-mode handle: low = FP32 arithmetic, high = FP64
static void enqueue_poly_map(const bjac_handle *M, int high, PcgState *st, const double *r, double *z, double *part,
                             hipStream_t s) {
  const PolyArgs a = poly_args(M, st, high);
  if (high || !M->plow)
    enqueue_poly_app<double>(M, a, r, z, part, s);
  else
    enqueue_poly_app<float>(M, a, r, z, part, s);
}

// ---------------------------------------------------------------- launchers
int launch_off16(int n, const int32_t *rp, const int32_t *ci, int16_t *o, int32_t *flag, hipStream_t s) {
  hipLaunchKernelGGL(off16_kernel, dim3(poly_grid(n)), dim3(256), 0, s, n, rp, ci, o, flag);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}

// The 8-bit value codes live in the compact-index region after the 8-bit
// column codes, from the first 16-byte boundary at or after nnz bytes (the
// region holds nnz + 16 int16 slots: room for both).
static const uint8_t *value_codes(const int16_t *o16, int64_t nnz) {
  return (const uint8_t *)o16 + ((nnz + 15) & ~(int64_t)15);
}

static void launch_spmv(const bjac_csr *A, const double *z, const double *pold, double *pnew, double *q,
                        PcgState *st, double *part, int mode, hipStream_t s, const int16_t *o16 = nullptr,
                        const double *rv = nullptr, const int *dict = nullptr, bool nt = false,
                        const double *vdict = nullptr) {
  SpmvArgs a{};
  a.rv = rv;
  a.o16 = o16;
  a.dict = dict;
  a.v8 = o16 ? value_codes(o16, A->nnz) : nullptr;
  a.vdict = vdict;
  a.n = (int32_t)A->n;
  a.ntiles = (int)((A->n + kSpmvRows - 1) / kSpmvRows);
  a.rp = A->row_ptr;
  a.ci = A->col_idx;
  a.v = A->val;
  a.z = z;
  a.pold = pold;
  a.pnew = pnew;
  a.q = q;
  a.st = st;
  a.part = part;
  a.nnz8 = (int32_t)(A->nnz & ~(int64_t)7);
  a.nnz16 = (int32_t)(A->nnz & ~(int64_t)15);
  const uintptr_t al = (uintptr_t)A->val | (uintptr_t)A->col_idx | (uintptr_t)o16;
  a.vec = (al & 15) == 0;
  if (mode == SPMV_PCG && nt) {
    const void *k = (const void *)spmv_kernel<SPMV_PCG, true>;
    hipLaunchKernelGGL((spmv_kernel<SPMV_PCG, true>), dim3(grid_for_waves(a.ntiles, k)), dim3(256), 0, s, a);
  } else if (mode == SPMV_PCG) {
    const void *k = (const void *)spmv_kernel<SPMV_PCG>;
    hipLaunchKernelGGL(spmv_kernel<SPMV_PCG>, dim3(grid_for_waves(a.ntiles, k)), dim3(256), 0, s, a);
  } else if (mode == SPMV_CG && nt) {
    const void *k = (const void *)spmv_kernel<SPMV_CG, true>;
    hipLaunchKernelGGL((spmv_kernel<SPMV_CG, true>), dim3(grid_for_waves(a.ntiles, k)), dim3(256), 0, s, a);
  } else if (mode == SPMV_CG) {
    const void *k = (const void *)spmv_kernel<SPMV_CG>;
    hipLaunchKernelGGL(spmv_kernel<SPMV_CG>, dim3(grid_for_waves(a.ntiles, k)), dim3(256), 0, s, a);
  } else {
    const void *k = (const void *)spmv_kernel<SPMV_PLAIN>;
    hipLaunchKernelGGL(spmv_kernel<SPMV_PLAIN>, dim3(grid_for_waves(a.ntiles, k)), dim3(256), 0, s, a);
  }
}

struct MapSel {
  DevMap map;
  int prec;      // common precision, -1 if mixed
  bool fast;
  int64_t off0;
};

static MapSel sel_lo(const bjac_handle *h) {
  return MapSel{DevMap{h->ws, h->off_lo, h->scale_lo, h->tag_lo, h->w_lo, h->storage == BJAC_STORE_SYM},
                h->uprec_lo, h->fast_lo, h->lo_off0};
}
static MapSel sel_hi(const bjac_handle *h) {
  if (!h->off_hi) return sel_lo(h);
  return MapSel{DevMap{h->ws, h->off_hi, h->scale_hi, h->tag_hi, h->w_hi, h->storage == BJAC_STORE_SYM}, (int)P64,
                h->fast_hi, h->hi_off0};
}

template <class K>
static void launch_persistent(K kernel, hipStream_t s, const ApplyArgs &a, int per_cu_max = kGridPerCu) {
  hipLaunchKernelGGL(kernel, dim3(grid_for_waves(a.ntiles, (const void *)kernel, per_cu_max)), dim3(256), 0, s, a);
}

template <int B, int MODE, bool NT>
static void launch_fast_bmn(int prec, hipStream_t s, const ApplyArgs &a) {
  if constexpr (B >= 32 && MODE != M_UPD) {
    if (a.map.sym) {
      switch (prec) {
        case P64: launch_persistent(apply_fast_kernel<B, P64, MODE, true, NT>, s, a); break;
        case P32: launch_persistent(apply_fast_kernel<B, P32, MODE, true, NT>, s, a); break;
        case PBF16: launch_persistent(apply_fast_kernel<B, PBF16, MODE, true, NT>, s, a); break;
        default: launch_persistent(apply_fast_kernel<B, P16, MODE, true, NT>, s, a); break;
      }
      return;
    }
  }
  switch (prec) {
    case P64: launch_persistent(apply_fast_kernel<B, P64, MODE, false, NT>, s, a); break;
    case P32: launch_persistent(apply_fast_kernel<B, P32, MODE, false, NT>, s, a); break;
    case PBF16: launch_persistent(apply_fast_kernel<B, PBF16, MODE, false, NT>, s, a); break;
    default: launch_persistent(apply_fast_kernel<B, P16, MODE, false, NT>, s, a); break;
  }
}

// the streaming (non-temporal) variants exist for the modes of a PCG
// iteration, not for the standalone application
template <int B, int MODE>
static void launch_fast_bm(int prec, hipStream_t s, const ApplyArgs &a, bool nt) {
  if constexpr (MODE != M_APP) {
    if (nt) {
      launch_fast_bmn<B, MODE, true>(prec, s, a);
      return;
    }
  }
  launch_fast_bmn<B, MODE, false>(prec, s, a);
}

template <int MODE, int B>
static void launch_band_fast(int prec, hipStream_t s, const ApplyArgs &a) {
  switch (prec) {
    case P64: launch_persistent(apply_band_fast_kernel<B, MODE, P64>, s, a); break;
    case P32: launch_persistent(apply_band_fast_kernel<B, MODE, P32>, s, a); break;
    case PBF16: launch_persistent(apply_band_fast_kernel<B, MODE, PBF16>, s, a); break;
    case P16: launch_persistent(apply_band_fast_kernel<B, MODE, P16>, s, a); break;
    default: launch_persistent(apply_band_fast_kernel<B, MODE, -1>, s, a); break;
  }
}

// Band maps: the arithmetic tile path when every block but the last has the
// common padded size, else the setup's tile list.
template <int MODE>
static void launch_band(const bjac_handle *h, int prec, hipStream_t s, const ApplyArgs &a) {
  if (h->rows_uniform && h->uniform_b) {
    switch (h->uniform_b) {
      case 16: launch_band_fast<MODE, 16>(prec, s, a); break;
      case 32: launch_band_fast<MODE, 32>(prec, s, a); break;
      case 48: launch_band_fast<MODE, 48>(prec, s, a); break;
      default: launch_band_fast<MODE, 64>(prec, s, a); break;
    }
    return;
  }
  constexpr int G = kGridPerCuGeneric;
  switch (prec) {
    case P64: launch_persistent(apply_band_kernel<MODE, P64>, s, a, G); break;
    case P32: launch_persistent(apply_band_kernel<MODE, P32>, s, a, G); break;
    case PBF16: launch_persistent(apply_band_kernel<MODE, PBF16>, s, a, G); break;
    case P16: launch_persistent(apply_band_kernel<MODE, P16>, s, a, G); break;
    default: launch_persistent(apply_band_kernel<MODE, -1>, s, a, G); break;
  }
}

template <int MODE>
static void launch_mode(const bjac_handle *h, const MapSel &m, hipStream_t s, const ApplyArgs &a, bool nt) {
  if constexpr (MODE != M_UPD) {
    if (m.map.w) {
      launch_band<MODE>(h, m.prec, s, a);
      return;
    }
  }
  // the update-only mode reads no map: any fast instance serves
  const bool fast = MODE == M_UPD ? h->rows_uniform : m.fast;
  const int prec = MODE == M_UPD ? (int)P16 : m.prec;
  if (fast && h->uniform_b) {
    switch (h->uniform_b) {
      case 16: launch_fast_bm<16, MODE>(prec, s, a, nt); break;
      case 32: launch_fast_bm<32, MODE>(prec, s, a, nt); break;
      case 48: launch_fast_bm<48, MODE>(prec, s, a, nt); break;
      default: launch_fast_bm<64, MODE>(prec, s, a, nt); break;
    }
  } else if (MODE != M_APP && nt) {
    launch_persistent(apply_generic_kernel<MODE, true>, s, a, kGridPerCuGeneric);
  } else {
    launch_persistent(apply_generic_kernel<MODE>, s, a, kGridPerCuGeneric);
  }
}

// One launch of the application kernel in the given mode and map.
static void launch_apply(const bjac_handle *h, int mode, int want_high, const MapSel &m, double *x, double *r,
                         double *z, const double *p, const double *q, const double *rin, PcgState *st, double *part,
                         hipStream_t s, double *pw = nullptr, double *sw = nullptr, bool nt = false) {
  ApplyArgs a{};
  a.pw = pw;
  a.sw = sw;
  a.ntiles = h->ntiles;
  a.nb = h->nb;
  a.n = (int32_t)h->n;
  a.want_high = want_high;
  a.tile_blk = h->tile_blk;
  a.blk_row = h->blk_row;
  a.bpad = h->bpad;
  a.map = m.map;
  a.off0 = m.off0;
  a.x = x;
  a.r = r;
  a.z = z;
  a.p = p;
  a.q = q;
  a.rin = rin;
  a.st = st;
  a.part = part;
  switch (mode) {
    case M_FUSED: launch_mode<M_FUSED>(h, m, s, a, nt); break;
    case M_UPD: launch_mode<M_UPD>(h, m, s, a, nt); break;
    case M_APPDEV: launch_mode<M_APPDEV>(h, m, s, a, nt); break;
    case M_CG: launch_mode<M_CG>(h, m, s, a, nt); break;
    default: launch_mode<M_APP>(h, m, s, a, false); break;
  }
}

struct SolveWs {
  double *r, *z, *pa, *pb, *q, *part1, *part2, *part3;
  PcgState *st;
  int16_t *o16;   // [nnz + 16] row-relative column indices (or their 8-bit codes, then the value codes), or null
  int *dict;      // [256] the codes' dictionary, then the overflow flag
  double *vdict;  // [256] the value codes' dictionary, then the overflow flag (as int)
  size_t bytes;
};

static SolveWs carve_solve(void *ws, int64_t n, int64_t nnz16 = 0) {
  Carver c(ws);
  SolveWs w{};
  w.r = c.take<double>(n);
  w.z = c.take<double>(n);
  w.pa = c.take<double>(n);
  w.pb = c.take<double>(n);
  w.q = c.take<double>(n);
  w.part1 = c.take<double>(3 * kMaxGrid);  // spmv slots, then update/apply slot pairs
  w.part2 = w.part1 + kMaxGrid;
  w.part3 = c.take<double>(kMaxGrid);      // true-residual partials
  w.st = c.take<PcgState>(1);
  w.o16 = nnz16 > 0 ? c.take<int16_t>(nnz16 + 16) : nullptr;
  w.dict = nnz16 > 0 ? c.take<int>(kDictSize + 64) : nullptr;
  w.vdict = nnz16 > 0 ? c.take<double>(kDictSize + 8) : nullptr;
  w.bytes = c.used;
  return w;
}

// The handle's own stream for capturing its iteration graph (created on the
// first capture, destroyed with the handle): captures of distinct handles from
// distinct threads never share a stream.
static hipStream_t capture_stream(bjac_handle *M) {
  if (!M->cap_stream && hipStreamCreateWithFlags(&M->cap_stream, hipStreamNonBlocking) != hipSuccess)
    M->cap_stream = nullptr;
  return M->cap_stream;
}

// The x / r update and the application: fused, or (adaptive switch) an update
// launch that decides the map and one application launch per map, of which
// only the chosen one does work. Events bracket the launches when given.
static void enqueue_update_apply(const bjac_handle *M, double *x, const SolveWs &w, bool temporal, const double *p,
                                 hipStream_t s, hipEvent_t *ev, bool nt = false) {
  if (M->kind == 1) {
    // the x / r update on 64-row wave tiles (the update mode of the block
    // application kernels, which reads no map)
    ApplyArgs ua{};
    ua.ntiles = (int32_t)((M->n + 63) / 64);
    ua.nb = ua.ntiles;
    ua.n = (int32_t)M->n;
    ua.x = x;
    ua.r = w.r;
    ua.p = p;
    ua.q = w.q;
    ua.st = w.st;
    ua.part = w.part2;
    if (ev) (void)hipEventRecord(ev[0], s);
    launch_persistent(apply_fast_kernel<64, P16, M_UPD>, s, ua);
    if (ev) (void)hipEventRecord(ev[1], s);
    if (temporal) {
      enqueue_poly_map(M, 1, w.st, w.r, w.z, w.part2, s);
      enqueue_poly_map(M, 0, w.st, w.r, w.z, w.part2, s);
    } else {
      enqueue_poly_map(M, 0, w.st, w.r, w.z, w.part2, s);
    }
    if (ev) (void)hipEventRecord(ev[2], s);
    return;
  }
  if (temporal) {
    if (ev) (void)hipEventRecord(ev[0], s);
    launch_apply(M, M_UPD, 0, sel_lo(M), x, w.r, w.z, p, w.q, nullptr, w.st, w.part2, s, nullptr, nullptr, nt);
    if (ev) (void)hipEventRecord(ev[1], s);
    launch_apply(M, M_APPDEV, 1, sel_hi(M), x, w.r, w.z, p, w.q, nullptr, w.st, w.part2, s, nullptr, nullptr, nt);
    launch_apply(M, M_APPDEV, 0, sel_lo(M), x, w.r, w.z, p, w.q, nullptr, w.st, w.part2, s, nullptr, nullptr, nt);
    if (ev) (void)hipEventRecord(ev[2], s);
  } else {
    if (ev) (void)hipEventRecord(ev[0], s);
    launch_apply(M, M_FUSED, 0, sel_lo(M), x, w.r, w.z, p, w.q, nullptr, w.st, w.part2, s, nullptr, nullptr, nt);
    if (ev) (void)hipEventRecord(ev[1], s);
  }
}

// The single-reduction iteration's update + application: p = u + beta p,
// s = w + beta s, x += alpha p, r -= alpha s, u = M^-1 r (u in z, w in q, p in
// pa, s in pb; p, s and u are updated in place: each row reads only itself).
static void enqueue_cg_apply(const bjac_handle *M, double *x, const SolveWs &w, hipStream_t s, hipEvent_t *ev,
                             bool nt = false) {
  if (ev) (void)hipEventRecord(ev[0], s);
  launch_apply(M, M_CG, 0, sel_lo(M), x, w.r, w.z, nullptr, w.q, nullptr, w.st, nullptr, s, w.pa, w.pb, nt);
  if (ev) (void)hipEventRecord(ev[1], s);
}

// Whether a PCG iteration streams: its SpMV and fused apply read at least the
// matrix (8-byte values, 1-byte column codes at best, row pointers), the
// stored inverses and 88 bytes per row of vectors. Beyond twice the 256 MiB
// last-level cache of the MI355X nothing is left there from one iteration to
// the next, and the kernels take the non-temporal variants (measured at
// 192^3, FP16 map, 1.5 GB per iteration: 316.9 -> 288.7 us per iteration);
// below it part of the data is found there again, and the hints lose it
// (128^3, FP16 map, 0.42 GB: 87.1 -> 94.6 us).
static bool streaming(const bjac_csr *A, const bjac_handle *M) {
  constexpr double kLastLevelCache = 256.0 * 1024 * 1024;
  const double bytes = (double)A->nnz * 9.0 + 4.0 * (double)(A->n + 1) + (double)M->low_bytes + 88.0 * (double)A->n;
  return bytes > 2.0 * kLastLevelCache;
}

// One PCG iteration: q = A p (p updated on the fly), then update + apply;
// single-reduction form: w = A u with the three dots, then update + apply.
static void enqueue_iteration(const bjac_csr *A, const bjac_handle *M, double *x, const SolveWs &w, bool temporal,
                              const double *pold, double *pnew, hipStream_t s, hipEvent_t *ev, bool cg, bool nt) {
  if (ev) (void)hipEventRecord(ev[0], s);
  if (cg) {
    launch_spmv(A, w.z, nullptr, nullptr, w.q, w.st, w.part1, SPMV_CG, s, w.o16, w.r, w.dict, nt, w.vdict);
    enqueue_cg_apply(M, x, w, s, ev ? ev + 1 : nullptr, nt);
    return;
  }
  launch_spmv(A, w.z, pold, pnew, w.q, w.st, w.part1, SPMV_PCG, s, w.o16, nullptr, w.dict, nt, w.vdict);
  enqueue_update_apply(M, x, w, temporal, pnew, s, ev ? ev + 1 : nullptr, nt);
}

// Profile mode: the same kernels launched one by one, bracketed by HIP events
// on the caller's stream. Only iterations that ran to their end are counted.
struct Prof {
  double t[3] = {0.0, 0.0, 0.0};  // spmv, apply (fused or split), update (split)
  int n[3] = {0, 0, 0};
};

static int profile_loop(const bjac_csr *A, const bjac_handle *M, double *x, const SolveWs &w, bool temporal,
                        int chunk, int max_launches, hipStream_t s, PcgState &hs, int &launches, Prof &prof,
                        bool cg, bool nt) {
  constexpr int EV = 4;  // events per iteration: spmv start, update/apply start, split point, end
  std::vector<hipEvent_t> ev((size_t)EV * chunk);
  // timing-only events: no system-scope cache writeback and invalidation at
  // each record, which would lengthen the bracketed kernel and cool the cache
  // for the next one (the captured iterations have no events between kernels)
  for (auto &e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return BJAC_EHIP;
  int rc = BJAC_OK;
  while (hs.status == ST_RUNNING && launches < max_launches) {
    const int it0 = hs.iter;
    for (int i = 0; i < chunk; ++i) {
      const bool even = (i & 1) == 0;
      enqueue_iteration(A, M, x, w, temporal, even ? w.pa : w.pb, even ? w.pb : w.pa, s, ev.data() + EV * i, cg, nt);
    }
    ++launches;
    if (hipMemcpyAsync(&hs, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = BJAC_EHIP;
      break;
    }
    const int done = hs.iter - it0;
    for (int i = 0; i < done && i < chunk; ++i) {
      hipEvent_t *e = ev.data() + EV * i;
      float a = 0.f, b = 0.f, c = 0.f;
      (void)hipEventElapsedTime(&a, e[0], e[1]);
      (void)hipEventElapsedTime(&b, e[1], e[2]);
      prof.t[0] += a;
      prof.n[0] += 1;
      if (temporal || M->kind == 1) {   // separate update and application launches
        (void)hipEventElapsedTime(&c, e[2], e[3]);
        prof.t[2] += b;
        prof.n[2] += 1;
        prof.t[1] += c;
        prof.n[1] += 1;
      } else {
        prof.t[1] += b;
        prof.n[1] += 1;
      }
    }
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  return rc;
}

}  // namespace mpb

using namespace mpb;

extern "C" int bjac_apply(const bjac_handle *h, int32_t which, const double *r, double *z, void *stream) {
  if (!h || !r || !z || r == z || (which != 0 && which != 1)) return BJAC_EINVAL;
  if (h->kind == 1) {
    enqueue_poly_map(h, which, nullptr, r, z, nullptr, (hipStream_t)stream);
    MPB_HIP(hipGetLastError());
    return BJAC_OK;
  }
  launch_apply(h, M_APP, 0, which == 1 ? sel_hi(h) : sel_lo(h), nullptr, nullptr, z, nullptr, nullptr, r, nullptr,
               nullptr, (hipStream_t)stream);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}

extern "C" int bjac_spmv(const bjac_csr *A, const double *p, double *q, void *stream) {
  if (!A || !p || !q || p == q || A->n < 1 || A->n >= (int64_t)1 << 31 || !A->row_ptr || !A->col_idx || !A->val)
    return BJAC_EINVAL;
  launch_spmv(A, p, nullptr, nullptr, q, nullptr, nullptr, SPMV_PLAIN, (hipStream_t)stream);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}

extern "C" int bjac_round(const double *in, void *out, int64_t count, int32_t prec, double scale, void *stream) {
  if (count < 0 || (count > 0 && (!in || !out)) || prec < BJAC_FP32 || prec > BJAC_FP16) return BJAC_EINVAL;
  int e;
  if (!(scale > 0) || std::frexp(scale, &e) != 0.5) return BJAC_EINVAL;
  return launch_round(in, out, count, prec, scale, (hipStream_t)stream);
}

extern "C" int pcg_workspace_query(int64_t n, size_t *workspace_bytes) {
  if (n < 1 || !workspace_bytes) return BJAC_EINVAL;
  *workspace_bytes = carve_solve(nullptr, n).bytes;
  return BJAC_OK;
}

extern "C" int pcg_workspace_query_csr(const bjac_csr *A, size_t *workspace_bytes) {
  if (!A || A->n < 1 || A->nnz < 0 || !workspace_bytes) return BJAC_EINVAL;
  *workspace_bytes = carve_solve(nullptr, A->n, A->nnz).bytes;
  return BJAC_OK;
}

// Checks shared by the PCG entry points; 0 or an error code.
static int check_solve(const bjac_csr *A, const bjac_handle *M, const double *b, double *x,
                       const bjac_solve_opts *opts) {
  if (!A || !M || !b || !x || !opts || b == x) return BJAC_EINVAL;
  if (A->n != M->n || !A->row_ptr || !A->col_idx || !A->val) return BJAC_EINVAL;
  if (!(opts->tol >= 0.0) || opts->maxit < 1) return BJAC_EINVAL;
  if (opts->variant != BJAC_PCG_TEXTBOOK && opts->variant != BJAC_PCG_SINGLE_REDUCTION) return BJAC_EINVAL;
  if (opts->cache_hints < BJAC_HINTS_AUTO || opts->cache_hints > BJAC_HINTS_STREAM) return BJAC_EINVAL;
  // the single-reduction form serves stored-inverse maps without the
  // adaptive switch (its update has no relres of the new residual yet)
  if (opts->variant == BJAC_PCG_SINGLE_REDUCTION && (M->policy.temporal != BJAC_TEMPORAL_NONE || M->kind != 0))
    return BJAC_EINVAL;
  return BJAC_OK;
}

// Events destroyed on every exit path.
struct EventPair {
  hipEvent_t e[2] = {nullptr, nullptr};
  ~EventPair() {
    for (auto &v : e)
      if (v) (void)hipEventDestroy(v);
  }
};

// The body of pcg_solve and pcg_solve_noalloc on a carved workspace.
// graphs: chunks of iterations replayed from a graph captured once per
// handle and argument set, timed with events; otherwise every chunk's
// kernels are launched directly and the time is taken on the host (no graph,
// event or allocation). Both launch the same kernels in the same order.
static int solve_run(const bjac_csr *A, bjac_handle *M, const double *b, double *x, const bjac_solve_opts *opts,
                     const SolveWs &w, const void *workspace, hipStream_t s, bool graphs, bjac_stats *stats) {
  const bool temporal = M->policy.temporal != BJAC_TEMPORAL_NONE;
  const bool cg = opts->variant == BJAC_PCG_SINGLE_REDUCTION;
  const bool nt = opts->cache_hints == BJAC_HINTS_STREAM || (opts->cache_hints == BJAC_HINTS_AUTO && streaming(A, M));
  int chunk = opts->chunk > 0 ? opts->chunk : 16;
  chunk += chunk & 1;  // even: the p buffers return to their roles

  EventPair ev;
  const auto h0 = std::chrono::steady_clock::now();
  if (graphs) {
    MPB_HIP(hipEventCreate(&ev.e[0]));
    MPB_HIP(hipEventCreate(&ev.e[1]));
    MPB_HIP(hipEventRecord(ev.e[0], s));
  }
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(1), 0, s, w.st, opts->tol, opts->maxit, M->policy.adp_tol,
                     M->policy.temporal, opts->relres_hist, opts->high_hist);
  if (w.o16) {
    // the compact copy of the column structure: 8-bit codes or 16-bit offsets
    const int n = (int)A->n, G = poly_grid(n);
    hipLaunchKernelGGL(dict_fill_kernel, dim3(1), dim3(kDictSize), 0, s, w.dict, w.dict + kDictSize);
    hipLaunchKernelGGL(dict_build_kernel, dim3(G), dim3(256), 0, s, n, A->row_ptr, A->col_idx, w.dict,
                       w.dict + kDictSize);
    hipLaunchKernelGGL(idx_encode_kernel, dim3(G), dim3(256), 0, s, n, A->row_ptr, A->col_idx, (const int *)w.dict,
                       (const int *)(w.dict + kDictSize), (uint8_t *)w.o16, w.o16, &w.st->cidx);
    // the value codes, after the 8-bit column codes, in the same region
    unsigned long long *vtab = (unsigned long long *)w.vdict;
    int *vovf = (int *)(w.vdict + kDictSize);
    hipLaunchKernelGGL(vdict_fill_kernel, dim3(1), dim3(kDictSize), 0, s, vtab, vovf);
    hipLaunchKernelGGL(vdict_build_kernel, dim3(G), dim3(256), 0, s, A->nnz, A->val, vtab, vovf);
    hipLaunchKernelGGL(val_encode_kernel, dim3(G), dim3(256), 0, s, A->nnz, A->val, (const unsigned long long *)vtab,
                       (const int *)vovf, (uint8_t *)value_codes(w.o16, A->nnz), (const int32_t *)&w.st->cidx);
    hipLaunchKernelGGL(vcode_commit_kernel, dim3(1), dim3(1), 0, s, (const int *)vovf, &w.st->cidx);
  }
  hipLaunchKernelGGL(pcg_fill_kernel, dim3(1024), dim3(256), 0, s, A->n, x, w.r, b, w.pa, w.q,
                     cg ? w.z : nullptr, cg ? w.pb : nullptr);
  hipLaunchKernelGGL(fill_empty_kernel, dim3(24), dim3(256), 0, s, w.part1, 3 * kMaxGrid);
  // first application z_0 = M^-1 r_0 (alpha = 0 leaves x = 0, r = b)
  if (cg) enqueue_cg_apply(M, x, w, s, nullptr);
  else enqueue_update_apply(M, x, w, temporal, w.pa, s, nullptr);
  MPB_HIP(hipGetLastError());

  // captured chunk of iterations, cached in the handle per argument set
  std::vector<uintptr_t> key;
  if (graphs && !opts->profile)
    key = {(uintptr_t)A->row_ptr, (uintptr_t)A->col_idx, (uintptr_t)A->val, (uintptr_t)A->n, (uintptr_t)x,
           (uintptr_t)workspace, (uintptr_t)chunk, (uintptr_t)w.o16, (uintptr_t)cg, (uintptr_t)nt};
  if (graphs && !opts->profile && (!M->gexec || M->gkey != key)) {
    if (M->gexec) {
      (void)hipGraphExecDestroy(M->gexec);
      M->gexec = nullptr;
    }
    hipStream_t cs = capture_stream(M);
    if (!cs) return BJAC_EHIP;
    MPB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    for (int i = 0; i < chunk; ++i) {
      const bool even = (i & 1) == 0;
      enqueue_iteration(A, M, x, w, temporal, even ? w.pa : w.pb, even ? w.pb : w.pa, cs, nullptr, cg, nt);
    }
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cs, &g) != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return BJAC_EHIP;
    }
    hipError_t ie = hipGraphInstantiate(&M->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      M->gexec = nullptr;
      return BJAC_EHIP;
    }
    M->gkey = key;
  }

  PcgState hs{};
  int launches = 0, restarts = 0;
  bool verified = false;
  const int max_launches = opts->maxit / chunk + 2;
  MPB_HIP(hipMemcpyAsync(&hs, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
  MPB_HIP(hipStreamSynchronize(s));
  Prof prof;
  if (opts->profile) {
    int rc = profile_loop(A, M, x, w, temporal, chunk, max_launches, s, hs, launches, prof, cg, nt);
    if (rc) return rc;
  } else {
    for (;;) {
      while (hs.status == ST_RUNNING && launches < max_launches + restarts) {
        if (graphs) {
          MPB_HIP(hipGraphLaunch(M->gexec, s));
        } else {
          for (int i = 0; i < chunk; ++i) {
            const bool even = (i & 1) == 0;
            enqueue_iteration(A, M, x, w, temporal, even ? w.pa : w.pb, even ? w.pb : w.pa, s, nullptr, cg, nt);
          }
          MPB_HIP(hipGetLastError());
        }
        ++launches;
        MPB_HIP(hipMemcpyAsync(&hs, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
        MPB_HIP(hipStreamSynchronize(s));
      }
      if (hs.status != ST_CONVERGED || !opts->verify) break;
      // FP64 check of the recursive residual: r = b - A x; restart if needed
      const int G = (int)std::min<int64_t>(kMaxGrid, std::max<int64_t>(1, (A->n + 255) / 256));
      hipLaunchKernelGGL(resid_kernel, dim3(G), dim3(256), 0, s, A->n, A->row_ptr, A->col_idx, A->val, x, b, w.r,
                         w.part3);
      hipLaunchKernelGGL(restart_kernel, dim3(1), dim3(256), 0, s, w.st, (const double *)w.part3, G);
      MPB_HIP(hipMemcpyAsync(&hs, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
      MPB_HIP(hipStreamSynchronize(s));
      verified = true;
      if (hs.status != ST_RUNNING || restarts >= opts->verify) {
        if (hs.status == ST_RUNNING) hs.status = ST_MAXIT;  // restarts exhausted: report not converged
        break;
      }
      ++restarts;
      if (cg) enqueue_cg_apply(M, x, w, s, nullptr);
      else enqueue_update_apply(M, x, w, temporal, w.pa, s, nullptr);
      MPB_HIP(hipGetLastError());
      MPB_HIP(hipMemcpyAsync(&hs, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
      MPB_HIP(hipStreamSynchronize(s));
    }
  }
  float ms = 0.f;
  if (graphs) {
    MPB_HIP(hipEventRecord(ev.e[1], s));
    MPB_HIP(hipEventSynchronize(ev.e[1]));
    (void)hipEventElapsedTime(&ms, ev.e[0], ev.e[1]);
  } else {
    MPB_HIP(hipStreamSynchronize(s));
    ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - h0).count();
  }
  int rc;
  switch (hs.status) {
    case ST_CONVERGED: rc = BJAC_OK; break;
    case ST_BREAKDOWN: rc = BJAC_EBREAKDOWN; break;
    case ST_SYNC_FAIL: rc = BJAC_EHIP; break;
    default: rc = BJAC_NOT_CONVERGED; break;
  }
  if (stats) {
    stats->iters = hs.iter < 0 ? 0 : hs.iter;
    stats->status = rc;
    stats->relres = hs.iter <= 0 ? (hs.status == ST_CONVERGED ? 0.0 : 1.0) : hs.relres;
    stats->rnorm0 = hs.rnorm0;
    stats->high_applications = hs.n_high;
    stats->graph_launches = launches;
    stats->solve_ms = ms;
    stats->spmv_ms = prof.t[0];
    stats->apply_ms = prof.t[1];
    stats->update_ms = prof.t[2];
    stats->n_spmv = prof.n[0];
    stats->n_apply = prof.n[1];
    stats->n_update = prof.n[2];
    stats->restarts = restarts;
    stats->true_relres = verified && hs.rnorm0 > 0.0 ? sqrt(hs.rr_true) / hs.rnorm0 : -1.0;
  }
  return rc;
}

extern "C" int pcg_solve(const bjac_csr *A, const bjac_handle *Mc, const double *b, double *x,
                         const bjac_solve_opts *opts, void *workspace, size_t workspace_bytes, bjac_stats *stats,
                         void *stream) {
  int rc = check_solve(A, Mc, b, x, opts);
  if (rc) return rc;
  if (!workspace) return BJAC_EINVAL;
  // with room for the 16-bit index copy the products use it, else the CSR's own
  SolveWs w = carve_solve(workspace, A->n, A->nnz);
  if (w.bytes > workspace_bytes || A->nnz < 1) w = carve_solve(workspace, A->n);
  if (w.bytes > workspace_bytes) return BJAC_ENOMEM;
  return solve_run(A, const_cast<bjac_handle *>(Mc), b, x, opts, w, workspace, (hipStream_t)stream, true, stats);
}

// ---------------------------------------------------- no-allocation solve
// The PCG workspace of pcg_solve_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends. Host code never passes its name to a
// kernel or a copy (on the host the name is only a stand-in): it uses the
// device address hipGetSymbolAddress returns, taken once per device with that
// device current and kept in g_noalloc_ptr.
constexpr int64_t kNoAllocMaxRows = int64_t(1) << 20;
constexpr size_t kNoAllocBytes = ((5 * kNoAllocMaxRows + 4 * kMaxGrid) * sizeof(double) + sizeof(PcgState) +
                                  16 * 256 + 255) & ~size_t(255);
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

static std::mutex g_noalloc_mu;
static std::map<int, void *> g_noalloc_ptr;

static int noalloc_scratch(void **out) {
  int dev = 0;
  MPB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(dev);
  if (it == g_noalloc_ptr.end()) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BJAC_EHIP;
    it = g_noalloc_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return BJAC_OK;
}

extern "C" int pcg_solve_noalloc(const bjac_csr *A, const bjac_handle *Mc, const double *b, double *x,
                                 const bjac_solve_opts *opts, bjac_stats *stats, void *stream) {
  int rc = check_solve(A, Mc, b, x, opts);
  if (rc) return rc;
  if (opts->profile) return BJAC_EINVAL;          // profile mode creates events
  if (A->n > kNoAllocMaxRows) return BJAC_ENOMEM;  // beyond the static workspace
  void *ws = nullptr;
  if ((rc = noalloc_scratch(&ws))) return rc;
  const SolveWs w = carve_solve(ws, A->n);         // 32-bit column indices: no room for the 16-bit copy
  if (w.bytes > kNoAllocBytes) return BJAC_ENOMEM;
  return solve_run(A, const_cast<bjac_handle *>(Mc), b, x, opts, w, ws, (hipStream_t)stream, false, stats);
}
