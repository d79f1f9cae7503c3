// Host-side internals of libmpbjac: the handle, the device PCG state and the
// workspace carving shared by the setup and solver translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mpbjac.h"

namespace mpb {

constexpr int kWaveRows = 64;       // padded rows of one apply wave tile
constexpr int kSpmvRows = 64;       // rows of one SpMV wave tile
constexpr int kSpmvNnzCap = 448;    // CSR entries staged in LDS per batched SpMV wave tile
constexpr int kSpmvSlot = 512;      // LDS entries per wave of the PCG SpMV (16-byte chunks)
constexpr int kMaxGrid = 2048;      // persistent workgroups (multiple of 8)
constexpr int kGridPerCu = 2;       // persistent workgroups per compute unit (measured at 128^3:
                                    // 2 beats 3 by 3 us per FP16 apply, 1 loses 5 us per SpMV)
constexpr int kGridPerCuGeneric = 3;  // the same for the per-block dispatch applications (generic and
                                      // generic band) and the paper-mode CSR sweeps (measured: 2 per CU
                                      // costs the generic apply 8 %, the sweeps 20 %)

// Device-resident PCG scalars. Written only by the last workgroup of each
// kernel (ticket pattern) and by the init kernel.
struct alignas(64) PcgState {
  double rho;        // (r, z) of the current direction
  double pq;         // (p, A p)
  double alpha, beta;
  double rr;         // ||r||^2 after the last update
  double rz;
  double rnorm0;     // ||r_0|| = ||b||
  double relres;     // ||r|| / ||r_0|| seen by the next preconditioner application
  double tol, adp_tol;
  double rr_true;    // ||b - A x||^2 of the last verification
  int32_t iter;      // x updates done; -1 before the first application
  int32_t maxit;
  int32_t status;    // 0 running, 1 converged, 2 maxit, -3 breakdown
  int32_t cidx;      // compact column indices the SpMV reads (next to status:
                     // both come in one load): 0 none (the CSR's 32-bit
                     // indices), 1 16-bit col - row, 2 8-bit codes of col - row
  int32_t use_high;  // map for the next application (temporal switch)
  int32_t temporal;
  int32_t n_high;    // applications that used the FP64 map
  uint32_t ticket_a, ticket_b, ticket_c;
  int32_t restart;   // 1: the next application restarts CG from a replaced residual
  double *relres_hist;
  uint8_t *high_hist;
};

enum StateStatus { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXIT = 2, ST_BREAKDOWN = -3, ST_SYNC_FAIL = -4 };

// One stored precision map: byte offsets (from the workspace base) and scale
// of every block; band storage adds each block's half-bandwidth.
struct DevMap {
  const uint8_t *base;
  const int64_t *off;
  const double *scale;
  const uint8_t *tag;
  const uint8_t *w = nullptr;   // band storage: diagonals 0..w[k] kept; null: full blocks
  int32_t sym = 0;              // symmetric storage of the blocks of padded size 32..64
};

// Symmetric storage of a block of padded size B = 16 m (the inverse of an SPD
// block is symmetric): row tile I keeps only its columns 16 I .. B-1, stored
// as the single 16-row tile of a block of padded size B - 16 I in the full
// layout, strips back to back (I = 0 first). The quarters below the diagonal
// are the transposes of stored ones. Entries per block, and where strip I
// starts (elements of the block's format); for B = 16 this is full storage.
__host__ __device__ constexpr int sym_elems(int B) { return 128 * (B / 16) * (B / 16 + 1); }
__host__ __device__ constexpr int sym_strip_off(int B, int I) { return 256 * (I * (B / 16) - I * (I - 1) / 2); }
static_assert(sym_elems(32) == 768 && sym_strip_off(32, 1) == 512 && sym_elems(48) == 1536 &&
                  sym_elems(64) == 2560 && sym_strip_off(64, 3) == 256 * 9 && sym_elems(16) == 256,
              "symmetric layout sizes");

}  // namespace mpb

struct bjac_handle {
  int64_t n = 0;
  int32_t nb = 0;
  int32_t max_block = 0;
  int32_t ntiles = 0;
  bjac_policy policy{};
  hipStream_t stream = nullptr;
  uint8_t *ws = nullptr;
  size_t ws_bytes = 0;
  // device arrays inside the workspace
  int32_t *blk_row = nullptr;    // [nb+1]
  int32_t *tile_blk = nullptr;   // [ntiles+1] first block of each wave tile
  uint8_t *bpad = nullptr;       // [nb] padded block sizes
  int32_t uniform_b = 0;         // common padded size or 0
  int32_t uprec_lo = -1;         // common precision of the low map or -1
  // fast path: every block but the last has exactly uniform_b rows, the map
  // has one precision and stores block k at off0 + k * uniform_b^2 * bytes
  bool rows_uniform = false;
  bool fast_lo = false, fast_hi = false;
  int64_t lo_off0 = 0, hi_off0 = 0;
  int64_t *off_lo = nullptr, *off_hi = nullptr;
  double *scale_lo = nullptr, *scale_hi = nullptr;
  uint8_t *tag_lo = nullptr, *tag_hi = nullptr;
  // band storage (BJAC_STORE_BAND): half-bandwidth of every block per map
  int32_t storage = 0;
  uint8_t *w_lo = nullptr, *w_hi = nullptr;
  std::vector<uint8_t> h_w_lo, h_w_hi;
  float *feat = nullptr;         // [nb*16]
  int32_t *flags = nullptr;      // [nb] non-SPD marks
  int32_t max_row_nnz = 0;       // most entries in one row of the A given at setup
  // host copies
  std::vector<int32_t> h_blk_row;
  std::vector<uint8_t> h_bpad;
  std::vector<uint8_t> h_tag_lo;
  std::vector<int64_t> h_off_lo, h_off_hi;
  std::vector<double> h_scale_lo;
  int32_t hist[4] = {0, 0, 0, 0};
  int64_t low_bytes = 0, high_bytes = 0;
  // cached PCG graph and the stream it is captured on
  hipGraphExec_t gexec = nullptr;
  std::vector<uintptr_t> gkey;
  hipStream_t cap_stream = nullptr;
  // paper-mode BJAC(k, t) (kind 1): no stored inverses; k outer steps with t
  // point-Jacobi sweeps inside each block, in FP32 (low) or FP64
  int32_t kind = 0;
  int32_t pk = 1, pt = 1, plow = 0;
  const int32_t *prp = nullptr, *pci = nullptr;   // A as given at setup (kept alive by the caller)
  const double *pval = nullptr;
  int64_t pnnz = 0;
  float *val32 = nullptr;        // [nnz] FP32 copy of A's values
  double *dinv64 = nullptr;      // [n] 1 / a_ii
  float *dinv32 = nullptr;       // [n]
  int32_t *rlo = nullptr, *rhi = nullptr;  // [n] column range of the row's block
  double *pbuf = nullptr;        // [6 n] work vectors of one application
};

namespace mpb {

// Bump allocator over a caller workspace; every piece 256-byte aligned.
struct Carver {
  uint8_t *base;
  size_t used = 0;
  explicit Carver(void *b) : base((uint8_t *)b) {}
  template <class T>
  T *take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T *p = base ? (T *)(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

#define MPB_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return BJAC_EHIP;             \
  } while (0)

// launchers implemented in solve.hip, used by setup and api
int launch_round(const double *in, void *out, int64_t count, int prec, double scale, hipStream_t s);
// writes col - row of every entry of the CSR as int16 into o; clears *flag
// when some entry lies more than 32767 rows from its row
int launch_off16(int n, const int32_t *rp, const int32_t *ci, int16_t *o, int32_t *flag, hipStream_t s);

}  // namespace mpb
