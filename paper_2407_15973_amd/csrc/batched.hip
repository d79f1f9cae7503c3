// Batched multi-right-hand-side block-Jacobi PCG: many independent SPD systems
// (stacked into one block-diagonal CSR) with 1..8 right-hand sides each; every
// (system, column) pair runs its own CG (Sec. 3.2) with its own scalars and
// stops on its own relative residual (Sec. 4.2). The block products
// Z_blk = s * Hhat R_blk (Algorithm 3.1 applied to up to 8 columns at once)
// run on the matrix cores: the stored fragment layout is the A operand of the
// 16x16x4 FP32 (and FP64) matrix instructions, the FP32 copies of the
// residual columns form the B operand.
//
// Each kernel walks fixed chunks of rows (SpMV) or of whole blocks (apply)
// that never cross a system; per-chunk, per-column partial dots are reduced
// per system by a one-workgroup-per-system kernel in chunk order, so results
// are deterministic and no intra-kernel cross-workgroup synchronisation is
// needed.
#include <math.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace mpb {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kBCols = 8;          // most right-hand sides per system
constexpr int kBWaveRows = 64;

enum BStatus { BS_RUNNING = 0, BS_CONVERGED = 1, BS_MAXIT = 2, BS_BREAKDOWN = -3 };

struct BTables {
  int32_t S, nch, nach;
  const int32_t *sys_row, *sys_m, *sys_col, *sys_ach;
  const int32_t *sys_ch;     // SpMV chunks of system s: [sys_ch[s], sys_ch[s+1]), sys_rpc[s] rows each
  const int32_t *sys_rpc;    // rows per SpMV chunk of system s (floor(64 / m), fewer for long rows)
  const int64_t *sys_vec;    // system start in the solver's vectors (64-byte aligned)
  const int64_t *sys_xvec;   // system start in the caller's b and x (contiguous)
  const int32_t *ach_blk, *ach_sys;   // apply chunks: blocks [ach_blk[i], ach_blk[i+1])
};

struct BState {
  double *rho, *alpha, *beta, *rnorm0, *relres;
  int32_t *iter, *status;
  int32_t *n_active;
  double tol;
  int32_t maxit;
};

__device__ __forceinline__ void bwave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ SpMV
// q = A p with p = z + beta p_old formed at every read (the direction update
// of PCG fused into the product), p_new and q written, (p, q) per column.
//
// Work unit: a chunk of one system's rows with at most 64 (row, column)
// elements, floor(64 / m) rows of a system with m columns (fewer when the
// longest row of A would overflow the chunk's LDS slot). Lane l owns
// element (l / m, l mod m), so consecutive lanes touch consecutive doubles of
// the row-major [rows][m] vectors, and one pass of the wave covers the chunk.
// Chunks are numbered system by system; the chunk range is cut into 8 runs of
// about equal cost, one per XCD (workgroup g runs on XCD g mod 8).
//
// Order: the waves of an XCD take the chunks of its run in increasing order
// from one counter (an atomic grab of `grab_k` chunks at a time), so the
// chunks in flight on an XCD form one narrow window of consecutive rows, and
// the rows a gather needs one grid plane away were fetched into that XCD's L2
// moments earlier by another wave. (With a fixed round-robin split the waves
// drift apart, the rows in flight spread far beyond what the L2 holds, and the
// neighbour reads fetch the same rows from memory several times over.)
//
// Software pipeline, one chunk per step: chunk i's gathers of z and p_old are
// issued after chunk i+1's CSR loads (16-byte chunks into registers), chunk
// i+2's row-pointer loads, the next grab and chunk i-1's stores (held back a
// step), so all of them share one round trip and nothing is left in flight
// when the step ends. A chunk's geometry follows from per-system tables kept
// in scalar registers, re-read only when a chunk lies in a later system.
constexpr int kBSlot = 512;   // LDS entries per wave: a chunk's CSR window in 16-byte chunks

struct BSpmvArgs {
  BTables t;
  const int32_t *rp, *ci;
  const double *v;
  const double *z, *pold;
  double *pnew, *q;
  const double *beta;
  double *part;              // (p, q) of system s's chunk k, column c: part[sys_pbase[s] + k m + c]
  const int32_t *sys_pbase;  // [S + 1]
  const int32_t *n_active;
  const int32_t *sched;      // [9] chunk run of each XCD
  const int32_t *run_sys;    // [8] system of each run's first chunk
  int32_t *grab;             // [8 * 32] chunk counter of each run (one per 128 bytes)
  int32_t grab_k;            // chunks per grab
  const int16_t *o16;        // col - row of every entry (16-bit copy; kernel REL = true)
  int32_t nnz;
};

struct SpmvLds {
  __align__(16) double v[kBSlot];
  __align__(16) int c[kBSlot];   // 32-bit indices, or the 16-bit copy in the first half
  int rp[65];
};

using bu32x4 = unsigned int __attribute__((ext_vector_type(4)));

// floor(e / m) for 0 <= e < 4096 and 1 <= m <= 8 (multiply by ceil(2^16/m);
// the rounding error e / 2^16 stays below 1/8)
__device__ __forceinline__ int div_small(int e, int m) {
  const int inv = (65536 + m - 1) / m;
  return (e * inv) >> 16;
}

// The system a wave is in (wave-uniform).
struct BSysState {
  int32_t s, chs, che;   // system and its chunks [chs, che)
  int32_t rs, nrows, m, R, c0, pbase;   // R: rows per chunk
  int64_t vsys;          // start of its block in the solver's vectors
};

// Every field is moved into a scalar register as it is loaded, so the wait
// for these loads stays inside the (rare) branch that fetches a new system:
// values left in vector registers would make the compiler wait for them at
// their first use after the branches join, on every step, and that wait
// would also drain the next chunk's loads issued in between.
__device__ __forceinline__ void bsys_fetch(const BSpmvArgs &a, int s, BSysState &y) {
  const int32_t *ch = a.t.sys_ch + s, *row = a.t.sys_row + s;
  y.s = s;
  y.chs = __builtin_amdgcn_readfirstlane(ch[0]);
  y.che = __builtin_amdgcn_readfirstlane(ch[1]);
  y.rs = __builtin_amdgcn_readfirstlane(row[0]);
  y.nrows = __builtin_amdgcn_readfirstlane(row[1]) - y.rs;
  y.m = __builtin_amdgcn_readfirstlane(a.t.sys_m[s]);
  y.R = __builtin_amdgcn_readfirstlane(a.t.sys_rpc[s]);
  y.c0 = __builtin_amdgcn_readfirstlane(a.t.sys_col[s]);
  y.pbase = __builtin_amdgcn_readfirstlane(a.sys_pbase[s]);
  const uint64_t v = (uint64_t)a.t.sys_vec[s];
  y.vsys = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
                     __builtin_amdgcn_readfirstlane((uint32_t)v));
}

// A chunk in the pipeline (wave-uniform): its index, first row and rows;
// ch = -1: none (the run is exhausted).
struct BSlot {
  int32_t ch = -1, r0 = 0, nr = 0;
};

// Moves a system cursor forward to the system holding chunk ch (chunk indices
// only grow along a run).
__device__ __forceinline__ void bsys_seek(const BSpmvArgs &a, int ch, BSysState &y) {
  while (ch >= y.che) bsys_fetch(a, y.s + 1, y);
}

__device__ __forceinline__ BSlot bslot_at(const BSpmvArgs &a, int ch, int ce, BSysState &y) {
  BSlot g;
  if (ch >= ce) return g;
  bsys_seek(a, ch, y);
  g.ch = ch;
  g.r0 = y.rs + (ch - y.chs) * y.R;
  g.nr = min(y.R, y.rs + y.nrows - g.r0);
  return g;
}

// Chunks of one run handed out in increasing order: `grab_k` at a time from
// the run's counter, the next grab in flight while the current ones are used.
struct BGrabber {
  int32_t *ctr;
  int cb, ce, K;
  int cur = 0, end = 0;
  int pend = 0;   // lane 0: result of the grab in flight
  // lane 0 takes the grab; the other lanes keep their (unused) value, so no
  // select joins the result before it is read
  __device__ __forceinline__ void issue() {
    if ((threadIdx.x & 63) == 0) pend = __hip_atomic_fetch_add(ctr, K, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // next chunk of the run, or ce once the run is exhausted (no grab after that)
  __device__ __forceinline__ int next() {
    if (cur >= end) {
      const int g = cb + __builtin_amdgcn_readfirstlane(pend);
      if (g >= ce) return ce;
      cur = g;
      end = min(g + K, ce);
      issue();
    }
    return cur++;
  }
};

// A wave-uniform pointer moved into scalar registers: the compiler then
// addresses p[lane] as scalar base + lane offset instead of keeping a per-lane
// 64-bit pointer alive across the loop.
// (The result is typed as a global-memory pointer: a pointer rebuilt from
// integers would otherwise be generic, and generic loads also wait on LDS.)
template <class T>
using gptr = __attribute__((address_space(1))) T *;

template <class T>
__device__ __forceinline__ gptr<T> wave_ptr(T *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gptr<T>)(((uint64_t)hi << 32) | lo);
}

template <bool REL>
__device__ __forceinline__ void bspmv_run(const BSpmvArgs &a, SpmvLds &L, int x) {
  constexpr int SL = kBSlot;
  constexpr int NV = SL * 8 / 16 / 64;               // value pieces per lane
  constexpr int NC = SL * (REL ? 2 : 4) / 16 / 64;   // index pieces per lane
  constexpr int EV = 2, EC = REL ? 8 : 4;            // entries per 16-byte piece
  constexpr int U = 7;                               // entries of a row with loads in flight together
  const int lane = threadIdx.x & 63;
  const int cb = a.sched[x], ce = a.sched[x + 1];
  if (cb >= ce) return;
  BSysState y, yX;   // cursors of the newest chunk and of the current one
  bsys_fetch(a, a.run_sys[x], y);
  yX = y;
  BGrabber gr{a.grab + 32 * x, cb, ce, a.grab_k};
  gr.issue();

  // end pointer of the lane's row in a chunk (lanes past the last row: the
  // chunk's end), and the chunk's first entry
  auto load_rp = [&](const BSlot &g, int &e0v) -> int {
    e0v = g.ch >= 0 ? a.rp[g.r0] : 0;
    return g.ch >= 0 ? a.rp[g.r0 + min(lane + 1, g.nr)] : 0;
  };
  // CSR window of a chunk: its first entry and count, and where its staged
  // 16-byte pieces start in each array (the first piece boundary at or below
  // the first entry; val is 8-byte, ci 4-byte aligned). The host caps the rows
  // of a chunk so that every window fits the LDS slot.
  const int vsh = (int)(((uintptr_t)a.v >> 3) & 1);   // val's offset from a 16-byte boundary (entries)
  const int csh = REL ? 0 : (int)(((uintptr_t)a.ci >> 2) & 3);
  auto window = [&](const BSlot &g, int rpl, int e0v, int &e0, int &cnt, int &bv, int &bc) {
    e0 = __builtin_amdgcn_readfirstlane(e0v);
    cnt = g.ch >= 0 ? __builtin_amdgcn_readlane(rpl, g.nr - 1) - e0 : 0;
    bv = e0 - ((e0 + vsh) & 1);
    bc = REL ? (e0 & ~7) : e0 - ((e0 + csh) & 3);
  };
  // 16-byte pieces of the window into registers; a piece that passes the end
  // of the arrays (the matrix's last chunk) is read entry by entry
  auto stage = [&](int e0, int cnt, int bv, int bc, bu32x4 (&gv)[NV], bu32x4 (&gc)[NC]) {
    const bu32x4 zero = {0u, 0u, 0u, 0u};
    const int end = e0 + cnt;
    const bu32x4 *vp = (const bu32x4 *)(a.v + bv);
    const bu32x4 *cp = REL ? (const bu32x4 *)(a.o16 + bc) : (const bu32x4 *)(a.ci + bc);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int c = lane + 64 * q;
      const int f = bv + c * EV;   // first entry of the piece
      gv[q] = zero;
      if (f < end) {
        if (f + EV <= a.nnz) {
          gv[q] = __builtin_nontemporal_load(vp + c);   // read once per product: do not displace the vectors
        } else {
          const uint64_t w = __double_as_longlong(a.v[f]);
          gv[q].x = (uint32_t)w;
          gv[q].y = (uint32_t)(w >> 32);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int c = lane + 64 * q;
      const int f = bc + c * EC;
      gc[q] = zero;
      if (f < end) {
        if (f + EC <= a.nnz) {
          gc[q] = __builtin_nontemporal_load(cp + c);
        } else {
          uint32_t w[4] = {0u, 0u, 0u, 0u};
          for (int j = 0; f + j < a.nnz && j < EC; ++j) {
            const uint32_t u = REL ? (uint32_t)(uint16_t)a.o16[f + j] : (uint32_t)a.ci[f + j];
            if (REL)
              w[j >> 1] |= u << (16 * (j & 1));
            else
              w[j] = u;
          }
          gc[q] = bu32x4{w[0], w[1], w[2], w[3]};
        }
      }
    }
  };

  // prologue: chunk X (current) with its CSR in registers, C with its row
  // pointers, R with its row-pointer loads in flight
  int e0vX, e0vC, e0vR;
  BSlot gX = bslot_at(a, gr.next(), ce, y);
  int rpX = load_rp(gX, e0vX);
  int e0X, cntX, bvX, bcX;
  window(gX, rpX, e0vX, e0X, cntX, bvX, bcX);
  bu32x4 gv[NV], gc[NC];
  stage(e0X, cntX, bvX, bcX, gv, gc);
  BSlot gC = bslot_at(a, gr.next(), ce, y);
  int rpC = load_rp(gC, e0vC);
  BSlot gR = bslot_at(a, gr.next(), ce, y);
  int rpR = load_rp(gR, e0vR);

  // stores of the previous chunk, issued in the next step: its values per
  // lane, its place from wave-uniform values
  int s_ch = -1, s_n = 0, s_m = 1;
  int64_t s_vb = 0, s_pb = 0;   // vector index of the chunk's first element, its first partial slot
  double s_q = 0.0, s_p = 0.0, s_pq = 0.0;
  auto flush = [&]() {
    if (s_ch < 0) return;
    if (lane < s_n) {   // non-temporal: read by the next launch only
      __builtin_nontemporal_store(s_q, &wave_ptr(a.q + s_vb)[lane]);
      __builtin_nontemporal_store(s_p, &wave_ptr(a.pnew + s_vb)[lane]);
    }
    if (lane < s_m) wave_ptr(a.part + s_pb)[lane] = s_pq;
  };

  while (gX.ch >= 0) {
    // (a) chunk X's CSR window and relative row pointers into LDS
    {
      const int nv = e0X + cntX - bvX, nc = e0X + cntX - bcX;   // staged entries
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const int c = lane + 64 * q;
        if (c * EV < nv) ((bu32x4 *)L.v)[c] = gv[q];
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int c = lane + 64 * q;
        if (c * EC < nc) ((bu32x4 *)L.c)[c] = gc[q];
      }
    }
    L.rp[lane + 1] = rpX - e0X;
    if (lane == 0) L.rp[0] = 0;
    bwave_lds_sync();
    // (b) chunk C: its window (row pointers arrived a step ago), CSR loads
    int e0C, cntC, bvC, bcC;
    window(gC, rpC, e0vC, e0C, cntC, bvC, bcC);
    bu32x4 hv[NV], hc[NC];
    stage(e0C, cntC, bvC, bcC, hv, hc);
    // (c) the chunk after R: rows (the grab arrived a step ago), row pointers;
    // the previous chunk's stores
    const BSlot gN = bslot_at(a, gr.next(), ce, y);
    int e0vN;
    const int rpN = load_rp(gN, e0vN);
    flush();
    // (d) chunk X: gathers, products and the per-column (p, q)
    bsys_seek(a, gX.ch, yX);
    const int m = yX.m;
    const int E = gX.nr * m;
    const bool has = lane < E;
    const int lr = div_small(lane, m);
    const int col = lane - lr * m;
    const int row = min(lr, gX.nr - 1);
    const int grow = gX.r0 + row;
    const int sidx = L.rp[row];
    const int len = has ? L.rp[row + 1] - sidx : 0;
    const double bt = a.beta[yX.c0 + col];
    const gptr<const double> zs = wave_ptr(a.z + yX.vsys);
    const gptr<const double> ps = wave_ptr(a.pold + yX.vsys);
    const int16_t *c16 = (const int16_t *)L.c + (e0X - bcX);
    const int *c32 = L.c + (e0X - bcX);
    const double *lv = L.v + (e0X - bvX);
    double acc = 0.0, prow = 0.0;
    bool found = false;
    for (int k0 = 0; k0 < len; k0 += U) {
      int cs[U];
      double gz[U], gp[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int e = sidx + min(k0 + k, len - 1);
        cs[k] = REL ? (int)c16[e] + grow : c32[e];
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        // a column outside the system (not a block-diagonal stack) is
        // clamped into it: wrong values for an invalid input, never an
        // access outside the vectors
        const int jl = min(max(cs[k] - yX.rs, 0), yX.nrows - 1);
        const uint32_t o = (uint32_t)(jl * m + col);
        gz[k] = zs[o];
        gp[k] = ps[o];
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        // the value is read once the gathers are in flight
        const double vv = lv[sidx + min(k0 + k, len - 1)];
        const double g = fma(bt, gp[k], gz[k]);
        acc = fma(k0 + k < len ? vv : 0.0, g, acc);
        const bool me = k0 + k < len && cs[k] == grow;
        prow = me ? g : prow;
        found = found || me;
      }
    }
    double prod = 0.0;
    if (has) {
      const uint32_t o = (uint32_t)((grow - yX.rs) * m + col);
      const double pr = found ? prow : fma(bt, ps[o], zs[o]);
      s_q = acc;
      s_p = pr;
      prod = pr * acc;
    }
    // column sums of pr * q over the chunk's rows: the lanes of one column
    // are congruent mod m, so for m a power of two a butterfly over the
    // strides >= m leaves column c's sum in lane c; otherwise through LDS
    bwave_lds_sync();   // every lane has read the CSR window
    if ((m & (m - 1)) == 0) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1)
        if (o >= m) prod += __shfl_xor(prod, o, 64);
    } else {
      L.v[lane] = prod;
      bwave_lds_sync();
      double t = 0.0;
      if (lane < m)
        for (int r = 0; r < gX.nr; ++r) t += L.v[lane + r * m];
      prod = t;
    }
    s_ch = gX.ch;
    s_n = E;
    s_m = m;
    s_vb = yX.vsys + (int64_t)(gX.r0 - yX.rs) * m;   // element l of the chunk is s_vb + l
    s_pb = yX.pbase + (int64_t)(gX.ch - yX.chs) * m;
    s_pq = prod;
    bwave_lds_sync();   // LDS free for the next chunk
    // shift the pipeline
    gX = gC;
    rpX = rpC;
    e0X = e0C;
    cntX = cntC;
    bvX = bvC;
    bcX = bcC;
#pragma unroll
    for (int q = 0; q < NV; ++q) gv[q] = hv[q];
#pragma unroll
    for (int q = 0; q < NC; ++q) gc[q] = hc[q];
    gC = gR;
    rpC = rpR;
    e0vC = e0vR;
    gR = gN;
    rpR = rpN;
    e0vR = e0vN;
  }
  flush();
}

// REL: the column structure is read as the 16-bit col - row copy. Four
// waves per SIMD (at most 128 registers, which the kernel fits without
// spilling; the compiler alone would take more and allow three).
template <bool REL>
__global__ __launch_bounds__(256, 4) void bspmv_kernel(BSpmvArgs a) {
  __shared__ SpmvLds lds[4];
  if (*a.n_active == 0) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  bspmv_run<REL>(a, lds[wv], blockIdx.x & 7);
}

// ---------------------------------------------------------- update + apply
struct BApplyArgs {
  BTables t;
  const int32_t *blk_row;
  const uint8_t *bpad;
  DevMap map;
  double *x, *r, *z;
  const double *p, *q;
  const double *alpha;
  double *part;          // [nach][2][8]: (r, r) then (r, z)
  const int32_t *n_active;
};

// One 16-row tile of a stored block times the FP32 (or FP64) residual columns
// in the wave's LDS, on the matrix cores; result rows written to zt[row][8].
template <int B, int P>
__device__ __forceinline__ void bmtile(const uint8_t *blk, double scale, int mt, const double *r64,
                                       double *zt, int lane) {
  constexpr int K = B / 4;
  constexpr int BY = prec_bytes(P);
  constexpr int V = 16 / BY;
  constexpr int G = (K + V - 1) / V;
  const int kq = lane >> 4, col = lane & 15;
  uint4 h[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int vg = layout_vg(B, V, g);
    const uint8_t *src = blk + (layout_group_base(B, V, mt, g) + (int64_t)lane * vg) * BY;
    if (vg * BY == 16) {
      h[g] = *(const uint4 *)src;
    } else {
      const uint2 t = *(const uint2 *)src;
      h[g] = make_uint4(t.x, t.y, 0u, 0u);
    }
  }
  if constexpr (P == P64) {
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int ks = 2 * g + e;
        const double av = e ? __hiloint2double((int)h[g].w, (int)h[g].z) : __hiloint2double((int)h[g].y, (int)h[g].x);
        const double bv = col < kBCols ? r64[(4 * ks + kq) * kBCols + col] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
    }
    // FP64 result layout: lane l, register j holds row 4j + l/16, column l%16
    if (col < kBCols) {
#pragma unroll
      for (int j = 0; j < 4; ++j) zt[(16 * mt + 4 * j + kq) * kBCols + col] = acc[j];
    }
  } else {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int vg = layout_vg(B, V, g);
      const uint32_t w[4] = {h[g].x, h[g].y, h[g].z, h[g].w};
#pragma unroll
      for (int e = 0; e < V; ++e) {
        if (e < vg) {
          const int ks = g * V + e;
          float av;
          if constexpr (P == P32) av = __uint_as_float(w[e]);
          else if constexpr (P == PBF16) av = (e & 1) ? bf16_hi(w[e >> 1]) : bf16_lo(w[e >> 1]);
          else av = (e & 1) ? f16_hi(w[e >> 1]) : f16_lo(w[e >> 1]);
          // the FP32 copy of r (Algorithm 3.1), rounded to nearest even
          const float bv = col < kBCols ? __double2float_rn(r64[(4 * ks + kq) * kBCols + col]) : 0.0f;
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
        }
      }
    }
    // FP32 result layout: lane l, register j holds row 4(l/16) + j, column l%16
    if (col < kBCols) {
#pragma unroll
      for (int j = 0; j < 4; ++j) zt[(16 * mt + 4 * kq + j) * kBCols + col] = (double)acc[j] * scale;
    }
  }
}

template <int B>
__device__ __forceinline__ void bmtile_dispatch(int prec, const uint8_t *blk, double scale, int mt,
                                                const double *r64, double *zt, int lane) {
  switch (prec) {
    case P64: bmtile<B, P64>(blk, scale, mt, r64, zt, lane); break;
    case P32: bmtile<B, P32>(blk, scale, mt, r64, zt, lane); break;
    case PBF16: bmtile<B, PBF16>(blk, scale, mt, r64, zt, lane); break;
    default: bmtile<B, P16>(blk, scale, mt, r64, zt, lane); break;
  }
}

// Z = s * Hhat R for one stored block of padded size B, tile by tile.
__device__ __forceinline__ void bblock(int B, int prec, const uint8_t *blk, double scale, const double *r64,
                                       double *zt, int lane) {
  for (int mt = 0; mt < B / 16; ++mt) {
    switch (B) {
      case 16: bmtile_dispatch<16>(prec, blk, scale, mt, r64, zt, lane); break;
      case 32: bmtile_dispatch<32>(prec, blk, scale, mt, r64, zt, lane); break;
      case 48: bmtile_dispatch<48>(prec, blk, scale, mt, r64, zt, lane); break;
      default: bmtile_dispatch<64>(prec, blk, scale, mt, r64, zt, lane); break;
    }
  }
}

// Band-stored blocks: block i keeps diagonals d = 0..w_i, diagonal d as B_i
// entries E_i(d, j) = H[j][j + d] (zero where j + d leaves the block). Lane lr
// owns LDS row lr (row li = lr - cb_i of block i) and forms, for every column c,
//   z = s_i (sum_{d<=w_i} E_i(d, li) r[lr + d][c] + sum_{1<=d<=w_i} E_i(d, li - d) r[lr - d][c])
// on the FP32 copy of r with FP32 accumulation (FP64 for FP64 blocks). A lane
// loads only its own E_i(d, li), once for all columns; E_i(d, li - d) is lane
// lr - d's value, moved across the wave (the tile's blocks sit on consecutive
// rows, so lane lr - d is in the same block exactly when li >= d). Eight
// diagonals a round, loaded as the 8-byte-aligned words holding the entries
// (every block starts on a 32-byte boundary and spans a multiple of 32 bytes)
// from positions clamped into the block, all in flight together.
__device__ __forceinline__ double bband_entry(uint2 w, int64_t bo, int prec) {
  const int b4 = (int)(bo & 7);
  const uint32_t w32 = (b4 & 4) ? w.y : w.x;
  const uint32_t h16 = (b4 & 2) ? (w32 >> 16) : (w32 & 0xffffu);
  if (prec == P64) return __hiloint2double((int)w.y, (int)w.x);
  if (prec == P32) return (double)__uint_as_float(w32);
  if (prec == PBF16) return (double)__uint_as_float(h16 << 16);
  return (double)f16_bits((uint16_t)h16);
}

template <int BP>
__device__ __forceinline__ void bband_tile(const BApplyArgs &a, int nk, const int (&cbo)[4], int cum, int M, int mB,
                                           int mtag, int64_t moff, double msc, int mw, const double *r64,
                                           const float *r32, double *zt, int lane) {
  constexpr int DC = 8;
  int Bv[4], tv[4], wv_[4];
  int64_t ov[4];
  double sv[4];
  int wmax = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int src = min(i, max(nk - 1, 0));
    Bv[i] = __builtin_amdgcn_readlane(mB, src);
    tv[i] = __builtin_amdgcn_readlane(mtag, src);
    wv_[i] = __builtin_amdgcn_readlane(mw, src);
    const int lo = __builtin_amdgcn_readlane((int)(moff & 0xffffffff), src);
    const int hi = __builtin_amdgcn_readlane((int)(moff >> 32), src);
    ov[i] = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    sv[i] = bcast(msc, src);
    if (i < nk) wmax = max(wmax, wv_[i]);
  }
  const int lr = lane;
  const bool mine = lr < cum;
  const int i = (lr >= cbo[1] && nk > 1) + (lr >= cbo[2] && nk > 2) + (lr >= cbo[3] && nk > 3);
  const int B = i == 0 ? Bv[0] : i == 1 ? Bv[1] : i == 2 ? Bv[2] : Bv[3];
  const int prec = BP >= 0 ? BP : (i == 0 ? tv[0] : i == 1 ? tv[1] : i == 2 ? tv[2] : tv[3]);
  const int w = mine ? (i == 0 ? wv_[0] : i == 1 ? wv_[1] : i == 2 ? wv_[2] : wv_[3]) : -1;
  const int64_t off = i == 0 ? ov[0] : i == 1 ? ov[1] : i == 2 ? ov[2] : ov[3];
  const double sc = i == 0 ? sv[0] : i == 1 ? sv[1] : i == 2 ? sv[2] : sv[3];
  const int cb = i == 0 ? cbo[0] : i == 1 ? cbo[1] : i == 2 ? cbo[2] : cbo[3];
  const int li = mine ? lr - cb : 0;
  const int wc = max(w, 0);
  const int BY = prec_bytes(prec);
  const bool f64 = prec == P64;
  const uint8_t *blk = a.map.base + off;
  using RT = std::conditional_t<BP == P64, uint64_t,
                                std::conditional_t<BP == P32, uint32_t, std::conditional_t<BP >= 0, uint16_t, uint2>>>;
  double acc64[kBCols];
  float acc32[kBCols];
#pragma unroll
  for (int c = 0; c < kBCols; ++c) {
    acc64[c] = 0.0;
    acc32[c] = 0.0f;
  }
  for (int d0 = 0; d0 <= wmax; d0 += DC) {
    RT hw[DC];
    int64_t hb[DC];
#pragma unroll
    for (int u = 0; u < DC; ++u) {
      hb[u] = ((int64_t)min(d0 + u, wc) * B + li) * BY;
      if constexpr (BP >= 0) hw[u] = *(const RT *)(blk + hb[u]);
      else hw[u] = *(const uint2 *)(blk + (hb[u] & ~(int64_t)7));
    }
#pragma unroll
    for (int u = 0; u < DC; ++u) {
      const int d = d0 + u;
      double ev;
      if constexpr (BP == P64) ev = __longlong_as_double((long long)hw[u]);
      else if constexpr (BP == P32) ev = (double)__uint_as_float(hw[u]);
      else if constexpr (BP == PBF16) ev = (double)__uint_as_float((uint32_t)hw[u] << 16);
      else if constexpr (BP == P16) ev = (double)f16_bits(hw[u]);
      else ev = bband_entry(hw[u], hb[u], prec);
      const double eh = (mine && d <= w) ? ev : 0.0;
      const double el = __shfl_up(eh, d, 64);
      const bool lower = mine && d >= 1 && li >= d;
      const int ru = min(lr + d, kBWaveRows - 1), rd = max(lr - d, 0);
      // all eight columns (columns >= M and padding rows are zero in LDS)
      if (f64) {
#pragma unroll
        for (int c = 0; c < kBCols; ++c) {
          acc64[c] = fma(eh, r64[ru * kBCols + c], acc64[c]);
          if (lower) acc64[c] = fma(el, r64[rd * kBCols + c], acc64[c]);
        }
      } else {
        const float4 *pu = (const float4 *)(r32 + ru * kBCols);
        const float4 *pd = (const float4 *)(r32 + rd * kBCols);
        const float4 u0 = pu[0], u1 = pu[1], w0 = pd[0], w1 = pd[1];
        const float ru8[kBCols] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
        const float rd8[kBCols] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        const float e32 = (float)eh, l32 = lower ? (float)el : 0.0f;
#pragma unroll
        for (int c = 0; c < kBCols; ++c) {
          acc32[c] = fmaf(e32, ru8[c], acc32[c]);
          acc32[c] = fmaf(l32, rd8[c], acc32[c]);
        }
      }
    }
  }
  if (mine) {
#pragma unroll
    for (int c = 0; c < kBCols; ++c)
      if (c < M) zt[lr * kBCols + c] = f64 ? acc64[c] : (double)acc32[c] * sc;
  }
}

__device__ __forceinline__ int rl(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ int64_t rl64(int64_t v, int src) {
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), src);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), src);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Blocks [k0, kend) of one system (rows from rs, vectors from v0, M columns).
// Per wave tile of consecutive whole blocks (<= 64 padded rows):
//  1. element phase: the tile's real rows are one contiguous run of
//     rows x M doubles; lane l takes elements l, l + 64, ... (UPD: x += alpha
//     p, r -= alpha q) and drops r (FP64) into LDS
//     at [padded row][column] (padding rows and columns >= M stay zero);
//  2. each 16-row tile of each block takes B/4 matrix-core steps with the
//     LDS columns as the B operand, results to LDS;
//  3. (r, r) and (r, z) per column from LDS: lane l takes column l mod 8;
//  4. element phase: z back to HBM, contiguous.
// BP: kFullBlocks (stored full blocks, matrix-core products), -1 (band
// storage, per-block precision) or the common precision of a band map.
constexpr int kFullBlocks = -2;

template <bool UPD, int BP>
__device__ __forceinline__ void bapply_blocks(const BApplyArgs &a, int k0, int kend, int rs, int64_t v0, int64_t xv0,
                                              int M, const double *alpha_g, double *r64, float *r32, double *zt,
                                              double &rr, double &rz) {
  const int lane = threadIdx.x & 63;
  // per element-slot column and alpha: element e = pass * 64 + lane has
  // column (e mod M); 64 mod M shifts it by the same amount every pass
  while (k0 < kend) {
    const int kl = min(k0 + min(lane, 4), kend);
    const int mB = kl < kend ? a.bpad[kl] : 0;
    const int mrow = a.blk_row[kl];
    const int kq = min(k0 + min(lane, 3), kend - 1);
    const int64_t moff = a.map.off[kq];
    const double msc = a.map.scale[kq];
    const int mtag = a.map.tag[kq];
    const int mw = BP != kFullBlocks ? (int)a.map.w[kq] : 0;
    int nk = 0, cum = 0;
    while (nk < 4 && k0 + nk < kend && cum + rl(mB, nk) <= kBWaveRows) {
      cum += rl(mB, nk);
      ++nk;
    }
    // block starts relative to the tile (rows) and in the padded LDS layout
    const int R0 = rl(mrow, 0);
    const int nreal = rl(mrow, nk) - R0;
    int bst[4], cbo[4];
    {
      int cb = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        bst[i] = i < nk ? rl(mrow, i) - R0 : (1 << 30);
        cbo[i] = cb;
        cb += i < nk ? rl(mB, i) : 0;
      }
    }
    // 1. zero this lane's LDS row, then the element phase
#pragma unroll
    for (int c = 0; c < kBCols; ++c) {
      r64[lane * kBCols + c] = 0.0;
      if constexpr (BP != kFullBlocks) r32[lane * kBCols + c] = 0.0f;
    }
    bwave_lds_sync();
    const int E = nreal * M;
    const int64_t base = v0 + (int64_t)(R0 - rs) * M;
    const int64_t xbase = xv0 + (int64_t)(R0 - rs) * M;
    for (int e = lane; e < E; e += 64) {
      const int row = div_small(e, M);
      const int c = e - row * M;
      double rv;
      if (UPD) {
        // non-temporal stores: read by later launches only (FP16 apply of the
        // 256-system batch: 5.18 -> 5.01 ms; non-temporal loads of p, q, x and
        // r as well made it slower, 5.33 ms)
        const double pv = a.p[base + e], qv = a.q[base + e], xv = a.x[xbase + e], r0v = a.r[base + e];
        const double al = alpha_g[c];
        __builtin_nontemporal_store(fma(al, pv, xv), a.x + xbase + e);
        rv = fma(-al, qv, r0v);
        __builtin_nontemporal_store(rv, a.r + base + e);
      } else {
        rv = a.r[base + e];
      }
      const int i = (row >= bst[1]) + (row >= bst[2]) + (row >= bst[3]);
      const int bs_i = i == 0 ? bst[0] : i == 1 ? bst[1] : i == 2 ? bst[2] : bst[3];
      const int cb_i = i == 0 ? cbo[0] : i == 1 ? cbo[1] : i == 2 ? cbo[2] : cbo[3];
      const int lr = row - bs_i + cb_i;
      r64[lr * kBCols + c] = rv;
      if constexpr (BP != kFullBlocks) r32[lr * kBCols + c] = __double2float_rn(rv);   // the FP32 copy of r
    }
    bwave_lds_sync();
    // 2. block products (band storage: row by row, all columns)
    if constexpr (BP != kFullBlocks) {
      bband_tile<BP>(a, nk, cbo, cum, M, mB, mtag, moff, msc, mw, r64, r32, zt, lane);
    } else {
      for (int i = 0; i < nk; ++i) {
        const int B = rl(mB, i);
        const int prec = rl(mtag, i);
        const uint8_t *blk = a.map.base + rl64(moff, i);
        const double sc = bcast(msc, i);
        const int cb = cbo[i];
        bblock(B, prec, blk, sc, r64 + cb * kBCols, zt + cb * kBCols, lane);
      }
    }
    bwave_lds_sync();
    // 3. per-column dots over the real rows of the tile: lane l sums column
    //    l mod 8 over LDS rows l / 8, l / 8 + 8, ...
    {
      const int c = lane & 7;
      for (int lr = lane >> 3; lr < cum; lr += 8) {
        const int li = (lr >= cbo[1] && nk > 1) + (lr >= cbo[2] && nk > 2) + (lr >= cbo[3] && nk > 3);
        const int lb_start = li == 0 ? cbo[0] : li == 1 ? cbo[1] : li == 2 ? cbo[2] : cbo[3];
        const int lb_rows = (li + 1 < nk ? (li == 0 ? bst[1] : li == 1 ? bst[2] : bst[3]) : nreal) -
                            (li == 0 ? bst[0] : li == 1 ? bst[1] : li == 2 ? bst[2] : bst[3]);
        if (c < M && lr - lb_start < lb_rows) {
          const double rv = r64[lr * kBCols + c];
          const double zv = zt[lr * kBCols + c];
          rr = fma(rv, rv, rr);
          rz = fma(rv, zv, rz);
        }
      }
    }
    // 4. z to HBM
    for (int e = lane; e < E; e += 64) {
      const int row = div_small(e, M);
      const int c = e - row * M;
      const int i = (row >= bst[1]) + (row >= bst[2]) + (row >= bst[3]);
      const int bs_i = i == 0 ? bst[0] : i == 1 ? bst[1] : i == 2 ? bst[2] : bst[3];
      const int cb_i = i == 0 ? cbo[0] : i == 1 ? cbo[1] : i == 2 ? cbo[2] : cbo[3];
      __builtin_nontemporal_store(zt[(row - bs_i + cb_i) * kBCols + c], a.z + base + e);
    }
    bwave_lds_sync();
    k0 += nk;
  }
}

template <int BP>
__device__ __forceinline__ void bapply_chunk(const BApplyArgs &a, int ch, int M, double *r64, float *r32,
                                             double *zt) {
  const int lane = threadIdx.x & 63;
  const int s = __builtin_amdgcn_readfirstlane(a.t.ach_sys[ch]);
  const int c0 = a.t.sys_col[s];
  double rr = 0.0, rz = 0.0;
  bapply_blocks<true, BP>(a, a.t.ach_blk[ch], a.t.ach_blk[ch + 1], a.t.sys_row[s], a.t.sys_vec[s], a.t.sys_xvec[s], M,
                      a.alpha + c0, r64, r32, zt, rr, rz);
  // column l mod 8 lives in lanes l, l + 8, ..., l + 56
#pragma unroll
  for (int o = 8; o < 64; o <<= 1) {
    rr += __shfl_xor(rr, o, 64);
    rz += __shfl_xor(rz, o, 64);
  }
  if (lane < kBCols) {
    a.part[(int64_t)ch * 2 * kBCols + lane] = rr;
    a.part[(int64_t)ch * 2 * kBCols + kBCols + lane] = rz;
  }
}

template <int BP>
__global__ __launch_bounds__(256) void bapply_kernel(BApplyArgs a) {
  constexpr bool BAND = BP != kFullBlocks;
  __shared__ double r64s[4][kBWaveRows * kBCols];
  __shared__ double zts[4][kBWaveRows * kBCols];
  __shared__ __align__(16) float r32s[BAND ? 4 : 1][BAND ? kBWaveRows * kBCols : 4];
  if (*a.n_active == 0) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // chunks round-robin over every wave of the grid, so that the waves of all
  // eight XCDs stream one window of the blocks at a time (contiguous
  // cost-balanced runs per wave took 5.63 ms against 5.25 ms per 256-system
  // sweep)
  for (int ch = (int)blockIdx.x * 4 + wv; ch < a.t.nach; ch += (int)gridDim.x * 4) {
    const int m = __builtin_amdgcn_readfirstlane(a.t.sys_m[a.t.ach_sys[ch]]);
    bapply_chunk<BP>(a, ch, m, r64s[wv], BAND ? r32s[BAND ? wv : 0] : nullptr, zts[wv]);
  }
}

// Z = M^-1 R for one n x m block of columns (no PCG): one wave per wave tile
// of the handle's partition, grid-stride.
template <int BP>
__global__ __launch_bounds__(256) void bapply_multi_kernel(BApplyArgs a, const int32_t *tile_blk, int ntiles,
                                                           int m) {
  constexpr bool BAND = BP != kFullBlocks;
  __shared__ double r64s[4][kBWaveRows * kBCols];
  __shared__ double zts[4][kBWaveRows * kBCols];
  __shared__ __align__(16) float r32s[BAND ? 4 : 1][BAND ? kBWaveRows * kBCols : 4];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double rr = 0.0, rz = 0.0;
  for (int t = blockIdx.x * 4 + wv; t < ntiles; t += gridDim.x * 4)
    bapply_blocks<false, BP>(a, tile_blk[t], tile_blk[t + 1], 0, 0, 0, m, nullptr, r64s[wv],
                               BAND ? r32s[BAND ? wv : 0] : nullptr, zts[wv], rr, rz);
}

// ------------------------------------------------------- per-system scalars
__device__ __forceinline__ double wg_sum(double v, double *sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__device__ __forceinline__ void freeze(BState &st, int col, int status) {
  st.status[col] = status;
  st.alpha[col] = 0.0;
  st.beta[col] = 0.0;
  atomicSub(st.n_active, 1);
}

// After the SpMV: alpha = rho / (p, A p) for every running column of system s.
// Other workgroups of the same launch decrement n_active, so the early-exit
// test reads it once per workgroup and shares the value: every thread of the
// workgroup then takes the same branch before the barriers of wg_sum.
__device__ __forceinline__ bool wg_none_active(const int32_t *n_active, int *flag) {
  if (threadIdx.x == 0) *flag = __hip_atomic_load(n_active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return *flag == 0;
}

// (p, q) per column from the SpMV's per-chunk partials, then alpha. One
// workgroup per segment of kBSegCh consecutive chunks of one system sums the
// segment's slots per column (coalesced: thread t reads the slots of column
// t mod m). A system with several segments publishes the segment totals with
// device-scope atomic stores into slots that hold kBEmpty and takes a ticket;
// the workgroup with the system's last ticket reads the totals with
// device-scope atomic loads (waiting for a slot whose store is still in
// flight), sums them in segment order and resets the slots and the ticket, so
// neither the result nor its rounding depends on which workgroup finishes
// first, and no cache maintenance is needed (device-scope atomics are
// coherent across the XCDs' L2 caches). Block 0 also rewinds the SpMV's
// chunk counters for the next launch (the SpMV of this iteration has ended:
// same stream).
constexpr int kBSegCh = 1024;                          // chunks per reduction segment
constexpr uint64_t kBEmpty = 0x7FF4D1CE0000BEEFull;    // signalling-NaN pattern no arithmetic produces
constexpr int kBSpinCap = 1 << 22;

struct BSegTabs {
  const int32_t *seg_sys;    // [nseg] system of each segment
  const int32_t *sys_seg;    // [S + 1] segments of system s: [sys_seg[s], sys_seg[s+1])
  const int32_t *sys_pbase;  // [S + 1] first partial slot of each system
  double *seg_part;          // [nseg * 8] column totals of each segment (kBEmpty when unused)
  uint32_t *sys_ticket;      // [S] segments of the system done (reset by the last)
};

// Fixed-order tree over the L / m partial sums of each column held in
// sh[c + j m] (j < L / m); column c's total ends in sh[c].
__device__ __forceinline__ void col_tree(double *sh, int L, int m) {
  const int t = (int)threadIdx.x;
  __syncthreads();
  for (int w = L / m; w > 1;) {
    const int h = w >> 1, nw = w - h;   // entries j < h take entry j + nw
    if (t < h * m) {
      const int c = t % m, j = t / m;
      sh[c + j * m] += sh[c + (j + nw) * m];
    }
    __syncthreads();
    w = nw;
  }
}

__global__ __launch_bounds__(256) void breduce_pq_kernel(BTables t, BState st, const double *part, BSegTabs sg,
                                                         int32_t *grab) {
  __shared__ double sh[256];
  __shared__ int act;
  __shared__ int last;
  const int tid = (int)threadIdx.x;
  if (blockIdx.x == 0 && tid < 8) grab[32 * tid] = 0;
  if (wg_none_active(st.n_active, &act)) return;
  const int seg = blockIdx.x;
  const int s = sg.seg_sys[seg];
  const int m = t.sys_m[s], c0 = t.sys_col[s];
  const int nk = t.sys_ch[s + 1] - t.sys_ch[s];
  const int k0 = (seg - sg.sys_seg[s]) * kBSegCh, k1 = min(nk, k0 + kBSegCh);
  // thread i < L (L: the largest multiple of m <= 256) sums the slots of
  // column i mod m with stride L
  {
    const double *v = part + sg.sys_pbase[s] + (int64_t)k0 * m;
    const int len = (k1 - k0) * m, L = 256 - 256 % m;
    double a[4] = {0.0, 0.0, 0.0, 0.0};   // four independent sums: four loads in flight
    if (tid < L) {
      int i = tid;
      for (; i + 3 * L < len; i += 4 * L)
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] += v[i + u * L];
      for (int u = 0; i < len; i += L, ++u) a[u] += v[i];
    }
    sh[tid] = (a[0] + a[1]) + (a[2] + a[3]);
    col_tree(sh, L, m);
  }
  double tot = tid < m ? sh[tid] : 0.0;
  const int nseg = sg.sys_seg[s + 1] - sg.sys_seg[s];
  if (nseg > 1) {
    if (tid < m)
      __hip_atomic_store((uint64_t *)(sg.seg_part + (int64_t)seg * 8 + tid), (uint64_t)__double_as_longlong(tot),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (tid == 0)
      last = __hip_atomic_fetch_add(sg.sys_ticket + s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
             (uint32_t)(nseg - 1);
    __syncthreads();
    if (!last) return;
    // segment totals in segment order: slot i of the system's [nseg][8]
    // block is column i mod 8
    // (loads of up to four slots issued together; only a slot still empty
    // is polled again)
    double a = 0.0;
    const int64_t b0 = (int64_t)sg.sys_seg[s] * 8;
    for (int i0 = tid; i0 < nseg * 8; i0 += 4 * 256) {
      uint64_t u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = i0 + 256 * k;
        u[k] = i < nseg * 8 && (i & 7) < m
                   ? __hip_atomic_load((uint64_t *)(sg.seg_part + b0 + i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   : 0ull;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = i0 + 256 * k;
        if (i >= nseg * 8 || (i & 7) >= m) continue;
        uint64_t *slot = (uint64_t *)(sg.seg_part + b0 + i);
        for (int spins = 0; u[k] == kBEmpty && spins < kBSpinCap; ++spins)
          u[k] = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(slot, kBEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a += u[k] == kBEmpty ? NAN : __longlong_as_double((long long)u[k]);   // never filled: poisons alpha
      }
    }
    sh[tid] = a;
    col_tree(sh, 256, 8);
    tot = tid < m ? sh[tid] : 0.0;
    if (tid == 0) __hip_atomic_store(sg.sys_ticket + s, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (tid < m) {
    const int col = c0 + tid;
    if (st.status[col] == BS_RUNNING) {
      if (!(tot > 0.0)) freeze(st, col, BS_BREAKDOWN);
      else st.alpha[col] = st.rho[col] / tot;
    }
  }
}

// After the update + apply: relres, convergence, beta, rho; init mode sets
// ||r_0|| and rho from the first application.
__global__ __launch_bounds__(256) void breduce_rz_kernel(BTables t, BState st, const double *part, int init) {
  __shared__ double sh[4];
  __shared__ int act;
  if (wg_none_active(st.n_active, &act)) return;
  const int s = blockIdx.x;
  const int m = t.sys_m[s], c0 = t.sys_col[s];
  const int cb = t.sys_ach[s], ce = t.sys_ach[s + 1];
  for (int c = 0; c < m; ++c) {
    double v1 = 0.0, v2 = 0.0;
    for (int ch = cb + (int)threadIdx.x; ch < ce; ch += 256) {
      v1 += part[(int64_t)ch * 2 * kBCols + c];
      v2 += part[(int64_t)ch * 2 * kBCols + kBCols + c];
    }
    const double rr = wg_sum(v1, sh);
    const double rz = wg_sum(v2, sh);
    if (threadIdx.x != 0) continue;
    const int col = c0 + c;
    if (st.status[col] != BS_RUNNING) continue;
    if (init) {
      st.rnorm0[col] = sqrt(rr);
      st.iter[col] = 0;
      if (st.rnorm0[col] == 0.0) {
        st.relres[col] = 0.0;
        freeze(st, col, BS_CONVERGED);
        continue;
      }
      if (!(rz > 0.0)) {
        freeze(st, col, BS_BREAKDOWN);
        continue;
      }
      st.rho[col] = rz;
      st.beta[col] = 0.0;
      continue;
    }
    st.iter[col] += 1;
    st.relres[col] = sqrt(rr) / st.rnorm0[col];
    if (st.relres[col] <= st.tol) {
      freeze(st, col, BS_CONVERGED);
    } else if (!(rz > 0.0)) {
      freeze(st, col, BS_BREAKDOWN);
    } else {
      st.beta[col] = rz / st.rho[col];
      st.rho[col] = rz;
      if (st.iter[col] >= st.maxit) freeze(st, col, BS_MAXIT);
    }
  }
}

// x = 0 and r = b per system (caller layout -> solver layout), p = q = 0,
// column state reset. blockIdx.y is the system.
__global__ __launch_bounds__(256) void binit_kernel(BTables t, double *x, double *r, const double *b, double *p,
                                                    double *q, int ncols, BState st, int32_t *grab, BSegTabs sg) {
  const int s = blockIdx.y;
  if (s == 0 && blockIdx.x == 0 && threadIdx.x < 8) grab[32 * threadIdx.x] = 0;   // SpMV chunk counters
  if (blockIdx.x == 0) {   // the system's reduction slots and ticket
    const int64_t b0 = (int64_t)sg.sys_seg[s] * 8, b1 = (int64_t)sg.sys_seg[s + 1] * 8;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) ((uint64_t *)sg.seg_part)[i] = kBEmpty;
    if (threadIdx.x == 0) sg.sys_ticket[s] = 0;
  }
  const int64_t xo = t.sys_xvec[s], vo = t.sys_vec[s];
  const int64_t len = t.sys_xvec[s + 1] - xo, plen = t.sys_vec[s + 1] - vo;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < plen; i += (int64_t)gridDim.x * 256) {
    if (i < len) {
      x[xo + i] = 0.0;
      r[vo + i] = b[xo + i];
    } else {
      r[vo + i] = 0.0;
    }
    p[vo + i] = 0.0;
    q[vo + i] = 0.0;
  }
  if (s == 0) {
    for (int c = blockIdx.x * 256 + threadIdx.x; c < ncols; c += gridDim.x * 256) {
      st.rho[c] = st.alpha[c] = st.beta[c] = st.rnorm0[c] = 0.0;
      st.relres[c] = INFINITY;
      st.iter[c] = 0;
      st.status[c] = BS_RUNNING;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *st.n_active = ncols;
  }
}

// ---------------------------------------------------------------- host side
constexpr int kBMaxGrid = 8192;               // workgroups of a batched launch

struct BPlan {
  int32_t S = 0, ncols = 0;
  int64_t nnz = 0;
  int64_t veclen = 0;
  std::vector<int32_t> sys_row, sys_m, sys_col, sys_ch, sys_rpc, sys_pbase, sys_seg, seg_sys, sys_ach, ach_blk,
      ach_sys;
  std::vector<int64_t> sys_vec, sys_xvec;
  int64_t xlen = 0;
  int32_t nch = 0, nslot = 0;                 // SpMV chunks and their partial (p, q) slots
  std::vector<int32_t> sched1, run_sys;       // [9] SpMV chunk run of each XCD, [8] system of its first chunk
};

static int make_bplan(const bjac_csr *A, const bjac_handle *M, int32_t S, const int32_t *sys_row,
                      const int32_t *sys_m, int apply_rows, BPlan &pl) {
  if (!M || S < 1 || !sys_row || !sys_m || sys_row[0] != 0 || sys_row[S] != M->n) return BJAC_EINVAL;
  if (M->kind != 0) return BJAC_EINVAL;  // stored block inverses only
  if (M->storage == BJAC_STORE_SYM) return BJAC_EINVAL;  // full or band storage only
  if (apply_rows < kBWaveRows || apply_rows > (1 << 20)) return BJAC_EINVAL;
  pl.S = S;
  pl.nnz = A ? A->nnz : 0;
  pl.sys_row.assign(sys_row, sys_row + S + 1);
  pl.sys_m.assign(sys_m, sys_m + S);
  pl.sys_col.resize(S + 1);
  pl.sys_vec.resize(S + 1);
  pl.sys_xvec.resize(S + 1);
  pl.sys_col[0] = 0;
  pl.sys_vec[0] = 0;
  pl.sys_xvec[0] = 0;
  for (int s = 0; s < S; ++s) {
    if (sys_row[s + 1] <= sys_row[s] || sys_m[s] < 1 || sys_m[s] > kBCols) return BJAC_EINVAL;
    pl.sys_col[s + 1] = pl.sys_col[s] + sys_m[s];
    const int64_t len = (int64_t)(sys_row[s + 1] - sys_row[s]) * sys_m[s];
    pl.sys_xvec[s + 1] = pl.sys_xvec[s] + len;
    pl.sys_vec[s + 1] = pl.sys_vec[s] + ((len + 7) & ~int64_t(7));
  }
  pl.ncols = pl.sys_col[S];
  pl.veclen = pl.sys_vec[S];
  pl.xlen = pl.sys_xvec[S];
  const double nnz_row = A && A->n > 0 ? (double)A->nnz / (double)A->n : 7.0;
  // SpMV chunks: floor(64 / m) rows of a system with m columns (at most 64
  // elements, one wave pass), fewer where the longest row of A would overflow
  // the chunk's LDS slot, numbered system by system; each chunk has m partial
  // (p, q) slots, a system's after those of the systems before it
  {
    const int cap = (kBSlot - 8) / std::max(1, M->max_row_nnz);   // rows whose entries surely fit
    if (cap < 1) return BJAC_EINVAL;   // a row with more entries than one slot holds
    pl.sys_ch.assign(1, 0);
    pl.sys_pbase.assign(1, 0);
    pl.sys_rpc.resize(S);
    std::vector<double> cost(S);   // modelled bytes of one chunk of each system
    int64_t nch = 0, nslot = 0;
    for (int s = 0; s < S; ++s) {
      const int m = sys_m[s], R = std::min(64 / m, cap);
      pl.sys_rpc[s] = R;
      const int64_t k = (sys_row[s + 1] - sys_row[s] + R - 1) / R;
      nch += k;
      nslot += k * m;
      if (nch >= ((int64_t)1 << 31) || nslot >= ((int64_t)1 << 31)) return BJAC_EINVAL;
      pl.sys_ch.push_back((int32_t)nch);
      pl.sys_pbase.push_back((int32_t)nslot);
      cost[s] = R * (nnz_row * 10.0 + 32.0 * m) + 8.0 * m + 64.0;
    }
    pl.nch = (int32_t)nch;
    pl.nslot = (int32_t)nslot;
    // reduction segments of kBSegCh chunks, never across systems
    pl.sys_seg.assign(1, 0);
    pl.seg_sys.clear();
    for (int s = 0; s < S; ++s) {
      const int k = (pl.sys_ch[s + 1] - pl.sys_ch[s] + kBSegCh - 1) / kBSegCh;
      pl.seg_sys.insert(pl.seg_sys.end(), k, s);
      pl.sys_seg.push_back((int32_t)pl.seg_sys.size());
    }
    // 8 runs of about equal modelled cost, one per XCD: run x starts at the
    // chunk where the cost prefix reaches x / 8 of the total
    double total = 0.0;
    for (int s = 0; s < S; ++s) total += (pl.sys_ch[s + 1] - pl.sys_ch[s]) * cost[s];
    pl.sched1.assign(9, 0);
    pl.sched1[8] = pl.nch;
    int s = 0;
    double pre = 0.0;   // cost of the systems before s
    for (int x = 1; x < 8; ++x) {
      const double goal = total * x / 8.0;
      while (s < S - 1 && pre + (pl.sys_ch[s + 1] - pl.sys_ch[s]) * cost[s] < goal) {
        pre += (pl.sys_ch[s + 1] - pl.sys_ch[s]) * cost[s];
        ++s;
      }
      int64_t c = pl.sys_ch[s] + (int64_t)std::llround((goal - pre) / cost[s]);
      c = std::min<int64_t>(std::max<int64_t>(c, pl.sys_ch[s]), pl.sys_ch[s + 1]);
      pl.sched1[x] = (int32_t)std::max<int64_t>(c, pl.sched1[x - 1]);
    }
    pl.run_sys.assign(8, S - 1);
    for (int x = 0; x < 8; ++x) {
      if (pl.sched1[x] >= pl.nch) continue;   // empty run: never read
      // the system whose chunk range holds the run's first chunk
      const auto it = std::upper_bound(pl.sys_ch.begin(), pl.sys_ch.end(), pl.sched1[x]);
      pl.run_sys[x] = (int32_t)(it - pl.sys_ch.begin()) - 1;
    }
  }
  // apply chunks: whole blocks, at most apply_rows padded rows, one system
  // each; every system boundary must be a block boundary
  const std::vector<int32_t> &br = M->h_blk_row;
  pl.sys_ach.assign(1, 0);
  int s = 0, rows = 0;
  bool fresh = true;
  for (int32_t k = 0; k < M->nb; ++k) {
    while (br[k] >= sys_row[s + 1]) {
      ++s;
      fresh = true;
      pl.sys_ach.push_back((int32_t)pl.ach_sys.size());
    }
    if (br[k + 1] > sys_row[s + 1]) return BJAC_EINVAL;  // block crosses systems
    const int B = M->h_bpad[k];
    if (fresh || rows + B > apply_rows) {
      pl.ach_blk.push_back(k);
      pl.ach_sys.push_back(s);
      rows = 0;
      fresh = false;
    }
    rows += B;
  }
  while ((int)pl.sys_ach.size() < S + 1) pl.sys_ach.push_back((int32_t)pl.ach_sys.size());
  pl.ach_blk.push_back(M->nb);
  return BJAC_OK;
}

// compute units of the current device and resident workgroups of the batched
// SpMV, queried once per device under a lock (handles may be used from
// several threads)
static std::mutex g_occ_mu;

static int cu_count() {
  static std::map<int, int> cus_of;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  auto it = cus_of.find(dev);
  if (it == cus_of.end()) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    it = cus_of.emplace(dev, cus).first;
  }
  return it->second;
}

// workgroups for `units` chunks: a multiple of 8 (XCD-ordered wave slots), at
// most wg_per_cu per compute unit, no more waves than chunks rounded up
static int bgrid(int units, int wg_per_cu) {
  int G = (units + 3) / 4;
  G = std::min(G, wg_per_cu * cu_count());
  G = std::min(G, kBMaxGrid);
  G = (G + 7) & ~7;
  return std::max(G, 8);
}

// workgroups of the SpMV that fit on one compute unit at once: its grid is at
// most one resident round (its waves loop until the counters run out)
static int spmv_resident(bool rel) {
  static std::map<std::pair<int, bool>, int> occ;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 2;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  auto it = occ.find({dev, rel});
  if (it == occ.end()) {
    int o = 0;
    const void *k = rel ? (const void *)bspmv_kernel<true> : (const void *)bspmv_kernel<false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k, 256, 0) != hipSuccess || o < 1) o = 2;
    it = occ.emplace(std::make_pair(dev, rel), o).first;
  }
  return it->second;
}

struct BWs {
  double *r, *z, *pa, *pb, *q, *part1, *part2;
  double *seg_part;        // [nseg * 8] SpMV reduction segment totals
  uint32_t *sys_ticket;    // [S]
  double *rho, *alpha, *beta, *rnorm0, *relres;
  int32_t *iter, *status, *n_active;
  int32_t *tabs;   // every int32 table, then both wave schedules
  int64_t *sys_vec, *sys_xvec;
  int16_t *o16;    // [nnz] 16-bit row-relative column indices
  int32_t *rel16;  // 1 while every entry fits 16 bits
  int32_t *grab;   // [8 * 32] SpMV chunk counter of each XCD run
  size_t bytes;
};

static size_t tabs_len(const BPlan &p) {
  return p.sys_row.size() + p.sys_m.size() + p.sys_col.size() + p.sys_ch.size() + p.sys_rpc.size() + p.sys_pbase.size() +
         p.sys_seg.size() + p.seg_sys.size() +
         p.sys_ach.size() + p.ach_blk.size() + p.ach_sys.size() + 9 + 8;
}

static BWs carve_b(void *ws, const BPlan &p) {
  Carver c(ws);
  BWs w{};
  w.r = c.take<double>(p.veclen);
  w.z = c.take<double>(p.veclen);
  w.pa = c.take<double>(p.veclen);
  w.pb = c.take<double>(p.veclen);
  w.q = c.take<double>(p.veclen);
  w.part1 = c.take<double>((size_t)p.nslot);
  w.seg_part = c.take<double>(p.seg_sys.size() * 8);
  w.sys_ticket = c.take<uint32_t>(p.S);
  w.part2 = c.take<double>((size_t)p.ach_sys.size() * 2 * kBCols);
  w.rho = c.take<double>(p.ncols);
  w.alpha = c.take<double>(p.ncols);
  w.beta = c.take<double>(p.ncols);
  w.rnorm0 = c.take<double>(p.ncols);
  w.relres = c.take<double>(p.ncols);
  w.iter = c.take<int32_t>(p.ncols);
  w.status = c.take<int32_t>(p.ncols);
  w.n_active = c.take<int32_t>(1);
  w.tabs = c.take<int32_t>(tabs_len(p));
  w.sys_vec = c.take<int64_t>(p.sys_vec.size());
  w.sys_xvec = c.take<int64_t>(p.sys_xvec.size());
  w.rel16 = c.take<int32_t>(1);
  w.grab = c.take<int32_t>(8 * 32);
  w.o16 = p.nnz > 0 ? c.take<int16_t>(p.nnz) : nullptr;
  w.bytes = c.used;
  return w;
}

// Everything one batched solve enqueues, built once per call.
struct BCtx {
  BPlan pl;
  BWs w{};
  BTables t{};
  BState st{};
  DevMap map{};
  int G1 = 8, G2 = 8;
  int grab_k = 1;
  bool rel = false;   // the SpMV reads the 16-bit col - row copy
  BSegTabs sg{};
  const int32_t *sched1 = nullptr, *run_sys = nullptr, *sys_pbase = nullptr;
  const bjac_csr *A = nullptr;
  const bjac_handle *M = nullptr;
  const double *b = nullptr;
  double *x = nullptr;
};

// defaults: the shape the autotuner picked for the 256-system workload
static void cfg_defaults(const bjac_batch_cfg *cfg, int &grab, int &wg_per_cu, int &spmv_wg, int &apply_rows) {
  grab = cfg && cfg->spmv_grab > 0 ? cfg->spmv_grab : 4;
  wg_per_cu = cfg && cfg->wg_per_cu > 0 ? cfg->wg_per_cu : 32;
  spmv_wg = cfg && cfg->spmv_wg_per_cu > 0 ? cfg->spmv_wg_per_cu : 32;
  apply_rows = cfg && cfg->apply_rows > 0 ? cfg->apply_rows : 256;
}

static bool cfg_valid(const bjac_batch_cfg *cfg) {
  return !cfg || (cfg->spmv_grab >= 0 && cfg->spmv_grab <= 64 && cfg->wg_per_cu >= 0 && cfg->wg_per_cu <= 32 &&
                  cfg->spmv_wg_per_cu >= 0 && cfg->spmv_wg_per_cu <= 32 && cfg->apply_rows >= 0);
}

static int bctx_make(const bjac_csr *A, const bjac_handle *M, int32_t nsys, const int32_t *sys_row,
                     const int32_t *sys_m, const double *b, double *x, double tol, int32_t maxit,
                     const bjac_batch_cfg *cfg, void *workspace, size_t workspace_bytes, hipStream_t s, BCtx &c) {
  if (!A || !M || !b || !x || !workspace || b == x || A->n != M->n) return BJAC_EINVAL;
  if (!(tol >= 0.0) || maxit < 1) return BJAC_EINVAL;
  if (!cfg_valid(cfg)) return BJAC_EINVAL;
  int grab, wg_per_cu, spmv_wg, apply_rows;
  cfg_defaults(cfg, grab, wg_per_cu, spmv_wg, apply_rows);
  c.grab_k = grab;
  int rc = make_bplan(A, M, nsys, sys_row, sys_m, apply_rows, c.pl);
  if (rc) return rc;
  c.w = carve_b(workspace, c.pl);
  if (c.w.bytes > workspace_bytes) return BJAC_ENOMEM;
  const BPlan &pl = c.pl;
  c.G2 = bgrid((int)pl.ach_sys.size(), wg_per_cu);
  // tables, uploaded once per call
  std::vector<int32_t> tabs;
  tabs.reserve(tabs_len(pl));
  auto put = [&](const std::vector<int32_t> &v) {
    const size_t o = tabs.size();
    tabs.insert(tabs.end(), v.begin(), v.end());
    return o;
  };
  const size_t o_row = put(pl.sys_row), o_m = put(pl.sys_m), o_col = put(pl.sys_col), o_ch = put(pl.sys_ch),
               o_rpc = put(pl.sys_rpc), o_pb = put(pl.sys_pbase), o_sseg = put(pl.sys_seg), o_segs = put(pl.seg_sys), o_ach = put(pl.sys_ach), o_ab = put(pl.ach_blk), o_as = put(pl.ach_sys),
               o_s1 = put(pl.sched1), o_rs = put(pl.run_sys);
  MPB_HIP(hipMemcpyAsync(c.w.tabs, tabs.data(), tabs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MPB_HIP(hipMemcpyAsync(c.w.sys_vec, pl.sys_vec.data(), pl.sys_vec.size() * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  MPB_HIP(hipMemcpyAsync(c.w.sys_xvec, pl.sys_xvec.data(), pl.sys_xvec.size() * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  const int32_t one = 1;
  MPB_HIP(hipMemcpyAsync(c.w.rel16, &one, sizeof(int32_t), hipMemcpyHostToDevice, s));
  // the host vectors above go out of scope at return: wait for the copies
  MPB_HIP(hipStreamSynchronize(s));
  // the 16-bit copy of the column structure the matrix-vector products read
  // (the SpMV kernel is chosen by whether every entry fits 16 bits)
  c.rel = false;
  if (c.w.o16 && A->n < ((int64_t)1 << 31)) {
    if ((rc = launch_off16((int)A->n, A->row_ptr, A->col_idx, c.w.o16, c.w.rel16, s))) return rc;
    int32_t fits = 0;
    MPB_HIP(hipMemcpyAsync(&fits, c.w.rel16, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MPB_HIP(hipStreamSynchronize(s));
    c.rel = fits != 0;
  }
  if (!c.rel) c.w.o16 = nullptr;
  c.G1 = bgrid(pl.nch, std::min(spmv_wg, spmv_resident(c.rel)));
  BTables &t = c.t;
  t.S = pl.S;
  t.nch = pl.nch;
  t.nach = (int32_t)pl.ach_sys.size();
  t.sys_row = c.w.tabs + o_row;
  t.sys_m = c.w.tabs + o_m;
  t.sys_col = c.w.tabs + o_col;
  t.sys_ch = c.w.tabs + o_ch;
  t.sys_rpc = c.w.tabs + o_rpc;
  t.sys_ach = c.w.tabs + o_ach;
  t.ach_blk = c.w.tabs + o_ab;
  t.ach_sys = c.w.tabs + o_as;
  t.sys_vec = c.w.sys_vec;
  t.sys_xvec = c.w.sys_xvec;
  c.sys_pbase = c.w.tabs + o_pb;
  c.sg = BSegTabs{c.w.tabs + o_segs, c.w.tabs + o_sseg, c.w.tabs + o_pb, c.w.seg_part, c.w.sys_ticket};
  c.sched1 = c.w.tabs + o_s1;
  c.run_sys = c.w.tabs + o_rs;
  c.st = BState{c.w.rho, c.w.alpha, c.w.beta, c.w.rnorm0, c.w.relres, c.w.iter, c.w.status, c.w.n_active, tol, maxit};
  c.map = DevMap{M->ws, M->off_lo, M->scale_lo, M->tag_lo, M->w_lo};
  c.A = A;
  c.M = M;
  c.b = b;
  c.x = x;
  return BJAC_OK;
}

static void benq_spmv_k(const BCtx &c, const double *pold, double *pnew, hipStream_t s) {
  BSpmvArgs a{};
  a.t = c.t;
  a.rp = c.A->row_ptr;
  a.ci = c.A->col_idx;
  a.v = c.A->val;
  a.z = c.w.z;
  a.pold = pold;
  a.pnew = pnew;
  a.q = c.w.q;
  a.beta = c.w.beta;
  a.part = c.w.part1;
  a.sys_pbase = c.sys_pbase;
  a.n_active = c.w.n_active;
  a.sched = c.sched1;
  a.run_sys = c.run_sys;
  a.grab = c.w.grab;
  a.grab_k = c.grab_k;
  a.o16 = c.w.o16;
  a.nnz = (int32_t)c.A->nnz;
  if (c.rel)
    hipLaunchKernelGGL(bspmv_kernel<true>, dim3(c.G1), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(bspmv_kernel<false>, dim3(c.G1), dim3(256), 0, s, a);
}

static void benq_spmv_r(const BCtx &c, hipStream_t s) {
  hipLaunchKernelGGL(breduce_pq_kernel, dim3((unsigned)c.pl.seg_sys.size()), dim3(256), 0, s, c.t, c.st,
                     (const double *)c.w.part1, c.sg, c.w.grab);
}

static void benq_spmv(const BCtx &c, const double *pold, double *pnew, hipStream_t s) {
  benq_spmv_k(c, pold, pnew, s);
  benq_spmv_r(c, s);
}

static void benq_apply_k(const BCtx &c, const double *p, hipStream_t s) {
  BApplyArgs a{};
  a.t = c.t;
  a.blk_row = c.M->blk_row;
  a.bpad = c.M->bpad;
  a.map = c.map;
  a.x = c.x;
  a.r = c.w.r;
  a.z = c.w.z;
  a.p = p;
  a.q = c.w.q;
  a.alpha = c.w.alpha;
  a.part = c.w.part2;
  a.n_active = c.w.n_active;
  if (!a.map.w) {
    hipLaunchKernelGGL(bapply_kernel<kFullBlocks>, dim3(c.G2), dim3(256), 0, s, a);
    return;
  }
  switch (c.M->uprec_lo) {
    case P64: hipLaunchKernelGGL(bapply_kernel<P64>, dim3(c.G2), dim3(256), 0, s, a); break;
    case P32: hipLaunchKernelGGL(bapply_kernel<P32>, dim3(c.G2), dim3(256), 0, s, a); break;
    case PBF16: hipLaunchKernelGGL(bapply_kernel<PBF16>, dim3(c.G2), dim3(256), 0, s, a); break;
    case P16: hipLaunchKernelGGL(bapply_kernel<P16>, dim3(c.G2), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(bapply_kernel<-1>, dim3(c.G2), dim3(256), 0, s, a); break;
  }
}

static void benq_apply_r(const BCtx &c, int init, hipStream_t s) {
  hipLaunchKernelGGL(breduce_rz_kernel, dim3(c.t.S), dim3(256), 0, s, c.t, c.st, (const double *)c.w.part2, init);
}

static void benq_apply(const BCtx &c, const double *p, int init, hipStream_t s) {
  benq_apply_k(c, p, s);
  benq_apply_r(c, init, s);
}

// x = 0, r = b, p = q = 0, then z_0 = M^-1 r_0 through the apply kernel with
// alpha = 0, which also yields ||r_0|| and rho_0
static void benq_init(const BCtx &c, hipStream_t s) {
  hipLaunchKernelGGL(binit_kernel, dim3(64, c.t.S), dim3(256), 0, s, c.t, c.x, c.w.r, c.b, c.w.pa, c.w.q,
                     c.pl.ncols, c.st, c.w.grab, c.sg);
  benq_apply(c, c.w.pa, 1, s);
}

// iteration j reads p from one buffer and writes the other
static void benq_iter(const BCtx &c, int j, hipStream_t s) {
  const bool even = (j & 1) == 0;
  benq_spmv(c, even ? c.w.pa : c.w.pb, even ? c.w.pb : c.w.pa, s);
  benq_apply(c, even ? c.w.pb : c.w.pa, 0, s);
}

static int bcollect(const BCtx &c, hipStream_t s, int32_t *col_iters, int32_t *col_status, double *col_relres,
                    bjac_stats *stats, int launches, float ms) {
  const int nc = c.pl.ncols;
  std::vector<int32_t> its(nc), sts(nc);
  std::vector<double> rel(nc);
  MPB_HIP(hipMemcpyAsync(its.data(), c.w.iter, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
  MPB_HIP(hipMemcpyAsync(sts.data(), c.w.status, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
  MPB_HIP(hipMemcpyAsync(rel.data(), c.w.relres, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
  MPB_HIP(hipStreamSynchronize(s));
  int worst = BJAC_OK, maxits = 0;
  double maxrel = 0.0;
  for (int i = 0; i < nc; ++i) {
    const int code = sts[i] == BS_CONVERGED ? BJAC_OK
                     : sts[i] == BS_BREAKDOWN ? BJAC_EBREAKDOWN
                                              : BJAC_NOT_CONVERGED;
    if (code == BJAC_EBREAKDOWN || (code == BJAC_NOT_CONVERGED && worst == BJAC_OK)) worst = code;
    if (col_iters) col_iters[i] = its[i];
    if (col_status) col_status[i] = code;
    if (col_relres) col_relres[i] = rel[i];
    maxits = std::max(maxits, its[i]);
    maxrel = std::max(maxrel, rel[i]);
  }
  if (stats) {
    const double sp = stats->spmv_ms, ap = stats->apply_ms, up = stats->update_ms;
    const int nsp = stats->n_spmv, nap = stats->n_apply, nup = stats->n_update;
    std::memset(stats, 0, sizeof(*stats));
    stats->iters = maxits;
    stats->status = worst;
    stats->graph_launches = launches;
    stats->solve_ms = ms;
    stats->relres = maxrel;
    stats->spmv_ms = sp;
    stats->apply_ms = ap;
    stats->update_ms = up;
    stats->n_spmv = nsp;
    stats->n_apply = nap;
    stats->n_update = nup;
  }
  return worst;
}

// Profile mode: eager launches, one host check of n_active per iteration,
// HIP events around every kernel on the caller's stream.
static int bcollect(const BCtx &c, hipStream_t s, int32_t *col_iters, int32_t *col_status, double *col_relres,
                    bjac_stats *stats, int launches, float ms);

static int bprofile_run(const BCtx &c, int maxit, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int32_t *col_iters,
                        int32_t *col_status, double *col_relres, bjac_stats *stats) {
  hipEvent_t ev[5];
  // timing-only events: no system-scope cache writeback and invalidation at each record
  for (auto &e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return BJAC_EHIP;
  int32_t active_h = 1;  // running columns, read back after every iteration
  int32_t *active = &active_h;
  double t_spmv = 0.0, t_apply = 0.0, t_red = 0.0;
  int n_it = 0, rc = BJAC_OK;
  if (hipMemcpyAsync(active, c.w.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = BJAC_EHIP;
  for (int j = 0; rc == BJAC_OK && *active > 0 && j < maxit; ++j) {
    const bool even = (j & 1) == 0;
    (void)hipEventRecord(ev[0], s);
    benq_spmv_k(c, even ? c.w.pa : c.w.pb, even ? c.w.pb : c.w.pa, s);
    (void)hipEventRecord(ev[1], s);
    benq_spmv_r(c, s);
    (void)hipEventRecord(ev[2], s);
    benq_apply_k(c, even ? c.w.pb : c.w.pa, s);
    (void)hipEventRecord(ev[3], s);
    benq_apply_r(c, 0, s);
    (void)hipEventRecord(ev[4], s);
    if (hipMemcpyAsync(active, c.w.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = BJAC_EHIP;
      break;
    }
    float a = 0.f, b = 0.f, d = 0.f, f = 0.f;
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[1], ev[2]);
    (void)hipEventElapsedTime(&d, ev[2], ev[3]);
    (void)hipEventElapsedTime(&f, ev[3], ev[4]);
    t_spmv += a;
    t_apply += d;
    t_red += b + f;
    ++n_it;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  MPB_HIP(hipEventRecord(e1, s));
  MPB_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (stats) {
    stats->spmv_ms = t_spmv;
    stats->apply_ms = t_apply;
    stats->update_ms = t_red;
    stats->n_spmv = stats->n_apply = n_it;
    stats->n_update = 2 * n_it;
  }
  return bcollect(c, s, col_iters, col_status, col_relres, stats, 0, ms);
}

}  // namespace mpb

using namespace mpb;

extern "C" int pcg_batched_workspace_query(const bjac_csr *A, const bjac_handle *M, int32_t nsys,
                                           const int32_t *sys_row, const int32_t *sys_m,
                                           const bjac_batch_cfg *cfg, size_t *workspace_bytes) {
  if (!workspace_bytes || !A || !cfg_valid(cfg)) return BJAC_EINVAL;
  int grab, wg_per_cu, spmv_wg, apply_rows;
  cfg_defaults(cfg, grab, wg_per_cu, spmv_wg, apply_rows);
  BPlan p;
  int rc = make_bplan(A, M, nsys, sys_row, sys_m, apply_rows, p);
  if (rc) return rc;
  *workspace_bytes = carve_b(nullptr, p).bytes;
  return BJAC_OK;
}

extern "C" int pcg_solve_batched(const bjac_csr *A, const bjac_handle *M, int32_t nsys, const int32_t *sys_row,
                                 const int32_t *sys_m, const double *b, double *x, const bjac_solve_opts *opts,
                                 const bjac_batch_cfg *cfg, void *workspace, size_t workspace_bytes,
                                 int32_t *col_iters, int32_t *col_status, double *col_relres, bjac_stats *stats,
                                 void *stream) {
  if (!opts || opts->variant != BJAC_PCG_TEXTBOOK) return BJAC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  BCtx c;
  int rc = bctx_make(A, M, nsys, sys_row, sys_m, b, x, opts->tol, opts->maxit, cfg, workspace, workspace_bytes, s, c);
  if (rc) return rc;
  int chunk = opts->chunk > 0 ? opts->chunk : 16;
  chunk += chunk & 1;  // an even count keeps the p ping-pong in step across launches

  hipEvent_t e0, e1;
  MPB_HIP(hipEventCreate(&e0));
  MPB_HIP(hipEventCreate(&e1));
  MPB_HIP(hipEventRecord(e0, s));
  benq_init(c, s);
  MPB_HIP(hipGetLastError());

  if (opts->profile) return bprofile_run(c, opts->maxit, s, e0, e1, col_iters, col_status, col_relres, stats);

  // capture `chunk` iterations once; kernels return at once when no column
  // is running, so replays past convergence cost only their launches
  hipStream_t cs = nullptr;
  MPB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return BJAC_EHIP;
  }
  for (int i = 0; i < chunk; ++i) benq_iter(c, i, cs);
  hipError_t ce = hipStreamEndCapture(cs, &g);
  if (ce == hipSuccess) ce = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (ce != hipSuccess) return BJAC_EHIP;

  int32_t active_h = 0;  // running columns, read back after every replay
  int32_t *active = &active_h;
  int launches = 0;
  const int max_launches = opts->maxit / chunk + 2;
  hipError_t le = hipMemcpyAsync(active, c.w.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess) le = hipStreamSynchronize(s);
  while (le == hipSuccess && *active > 0 && launches < max_launches) {
    le = hipGraphLaunch(ge, s);
    ++launches;
    if (le == hipSuccess) le = hipMemcpyAsync(active, c.w.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (le == hipSuccess) le = hipStreamSynchronize(s);
  }
  (void)hipGraphExecDestroy(ge);
  if (le != hipSuccess) return BJAC_EHIP;
  MPB_HIP(hipEventRecord(e1, s));
  MPB_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);

  if (stats) {
    stats->spmv_ms = stats->apply_ms = stats->update_ms = 0.0;
    stats->n_spmv = stats->n_apply = stats->n_update = 0;
  }
  return bcollect(c, s, col_iters, col_status, col_relres, stats, launches, ms);
}

extern "C" int pcg_batched_tune(const bjac_csr *A, const bjac_handle *M, int32_t nsys, const int32_t *sys_row,
                                const int32_t *sys_m, const double *b, double *x, const bjac_batch_cfg *cands,
                                int32_t ncand, int32_t iters, void *workspace, size_t workspace_bytes,
                                float *ms_per_iter, int32_t *best, void *stream) {
  if (!cands || ncand < 1 || iters < 1 || !best) return BJAC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  MPB_HIP(hipEventCreate(&e0));
  MPB_HIP(hipEventCreate(&e1));
  int bi = -1;
  float bms = 0.f;
  int rc = BJAC_OK;
  for (int k = 0; k < ncand && rc == BJAC_OK; ++k) {
    BCtx c;
    // tol = 0: no column stops during the timed iterations
    rc = bctx_make(A, M, nsys, sys_row, sys_m, b, x, 0.0, 1 << 30, &cands[k], workspace, workspace_bytes, s, c);
    if (rc) break;
    benq_init(c, s);
    benq_iter(c, 0, s);
    if (hipEventRecord(e0, s) != hipSuccess) rc = BJAC_EHIP;
    for (int j = 1; j <= iters && rc == BJAC_OK; ++j) benq_iter(c, j, s);
    if (rc == BJAC_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                          hipEventSynchronize(e1) != hipSuccess))
      rc = BJAC_EHIP;
    float ms = 0.f;
    if (rc == BJAC_OK) (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)iters;
    if (ms_per_iter) ms_per_iter[k] = ms;
    if (rc == BJAC_OK && (bi < 0 || ms < bms)) {
      bi = k;
      bms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  *best = bi;
  return BJAC_OK;
}

extern "C" int bjac_apply_multi(const bjac_handle *M, const double *R, double *Z, int32_t m, void *stream) {
  if (!M || !R || !Z || R == Z || m < 1 || m > kBCols) return BJAC_EINVAL;
  if (M->kind != 0 || M->storage == BJAC_STORE_SYM) return BJAC_EINVAL;
  BApplyArgs a{};
  a.blk_row = M->blk_row;
  a.bpad = M->bpad;
  a.map = DevMap{M->ws, M->off_lo, M->scale_lo, M->tag_lo, M->w_lo};
  a.r = const_cast<double *>(R);  // read only in this mode
  a.z = Z;
  const int G = std::max(1, std::min((M->ntiles + 3) / 4, 4 * cu_count()));
  hipStream_t st = (hipStream_t)stream;
  const int32_t *tb = (const int32_t *)M->tile_blk;
  if (!a.map.w) {
    hipLaunchKernelGGL(bapply_multi_kernel<kFullBlocks>, dim3(G), dim3(256), 0, st, a, tb, M->ntiles, (int)m);
  } else {
    switch (M->uprec_lo) {
      case P64: hipLaunchKernelGGL(bapply_multi_kernel<P64>, dim3(G), dim3(256), 0, st, a, tb, M->ntiles, (int)m); break;
      case P32: hipLaunchKernelGGL(bapply_multi_kernel<P32>, dim3(G), dim3(256), 0, st, a, tb, M->ntiles, (int)m); break;
      case PBF16:
        hipLaunchKernelGGL(bapply_multi_kernel<PBF16>, dim3(G), dim3(256), 0, st, a, tb, M->ntiles, (int)m);
        break;
      case P16: hipLaunchKernelGGL(bapply_multi_kernel<P16>, dim3(G), dim3(256), 0, st, a, tb, M->ntiles, (int)m); break;
      default: hipLaunchKernelGGL(bapply_multi_kernel<-1>, dim3(G), dim3(256), 0, st, a, tb, M->ntiles, (int)m); break;
    }
  }
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}
