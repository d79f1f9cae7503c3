// Block-Jacobi setup: extraction of the diagonal blocks A_ii from the CSR rows,
// FP64 inversion, block features, precision selection, scaling, correctly
// rounded downcast and packing (arXiv 2407.15973 Sec. 3.1 D_b; Sec. 3.2 and
// Algorithm 3.1 for the low-precision copy M^-1(p_l)).
#include <math.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace mpb {

enum TagMode { TAG_CONST = 0, TAG_RULE = 1, TAG_ARRAY = 2 };

struct SetupArgs {
  const int32_t *rp;
  const int32_t *ci;
  const double *val;
  const int32_t *blk_row;
  const int32_t *blist;   // blocks of this padded-size class
  int32_t nblist;
  int32_t tag_mode;
  int32_t tag_const;
  const uint8_t *tag_in;  // TAG_ARRAY
  uint8_t *tag_out;       // optional
  double theta, d16;
  float *feat;            // optional [nb*16]
  int32_t *flags;         // [nb] 1 = non-positive pivot
  int32_t *any_bad;
  uint8_t *base;          // workspace base for the arenas
  const int64_t *off_lo;  // pack the low map when non-null
  double *scale_lo;
  const int64_t *off_hi;  // pack the all-FP64 map when non-null
  double *scale_hi;
  // band storage: widths per format (first pass), chosen widths (packing pass)
  uint8_t *wband;         // [nb*4] when non-null: w of each format, indexed by Prec
  double band_rtol;       // <= 0: the format's unit roundoff
  const uint8_t *w_lo;    // packing: band store of the low map when non-null
  const uint8_t *w_hi;    // packing: band store of the all-FP64 map when non-null
  int32_t sym;            // packing: symmetric storage of the blocks of padded size 32..64
};

constexpr double kDomCap = 1e8;
constexpr double kGershFloor = 1e-16;
constexpr double kDomSlack = 1e-12;
constexpr int kScaleTopExp = 15;

template <int B, int P>
__device__ __forceinline__ void store_rows(uint8_t *dst, const double (&row)[B], int lane, double inv_s) {
  constexpr int K = B / 4;
  constexpr int V = 16 / prec_bytes(P);
  constexpr int G = (K + V - 1) / V;
  constexpr int BY = prec_bytes(P);
  const int mt = lane >> 4, r16 = lane & 15;
#pragma unroll
  for (int kq = 0; kq < 4; ++kq) {
    const int l = r16 + 16 * kq;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int vg = layout_vg(B, V, g);
      uint8_t *p = dst + (layout_group_base(B, V, mt, g) + (int64_t)l * vg) * BY;
      if constexpr (P == P64) {
        double2 v;
        v.x = row[4 * (g * V + 0) + kq];
        v.y = row[4 * (g * V + 1) + kq];
        *(double2 *)p = v;
      } else if constexpr (P == P32) {
        uint4 v;
        v.x = to_f32_bits(row[4 * (g * V + 0) + kq] * inv_s);
        v.y = to_f32_bits(row[4 * (g * V + 1) + kq] * inv_s);
        v.z = to_f32_bits(row[4 * (g * V + 2) + kq] * inv_s);
        v.w = to_f32_bits(row[4 * (g * V + 3) + kq] * inv_s);
        *(uint4 *)p = v;
      } else {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (e < vg) {
            const uint32_t bits = to_bits<P>(row[4 * (g * V + e) + kq] * inv_s);
            w[e >> 1] |= bits << (16 * (e & 1));
          }
        }
        if (vg == 8) {
          *(uint4 *)p = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
          *(uint2 *)p = make_uint2(w[0], w[1]);
        }
      }
    }
  }
}

// Symmetric storage of a block of padded size B (32, 48 or 64): the lane of
// row i (row tile I = i / 16) stores the columns 16 I .. B-1 of its row as row
// i % 16 of the single row tile of a block of padded size B - 16 I, at strip
// I's offset; the columns left of 16 I are the transposes of entries stored by
// the rows above.
template <int B, int P, int I>
__device__ __forceinline__ void store_sym_strip(uint8_t *dst, const double (&row)[B], int lane, double inv_s) {
  constexpr int W = B - 16 * I;
  double h[W];
#pragma unroll
  for (int j = 0; j < W; ++j) h[j] = row[16 * I + j];
  store_rows<W, P>(dst + (int64_t)sym_strip_off(B, I) * prec_bytes(P), h, lane - 16 * I, inv_s);
}

template <int B, int P>
__device__ __forceinline__ void store_rows_sym(uint8_t *dst, const double (&row)[B], int lane, double inv_s) {
  switch (lane >> 4) {
    case 0: store_sym_strip<B, P, 0>(dst, row, lane, inv_s); break;
    case 1: store_sym_strip<B, P, 1>(dst, row, lane, inv_s); break;
    case 2:
      if constexpr (B >= 48) store_sym_strip<B, P, 2>(dst, row, lane, inv_s);
      break;
    default:
      if constexpr (B >= 64) store_sym_strip<B, P, 3>(dst, row, lane, inv_s);
      break;
  }
}

// Stores block rows in the symmetric layout when it applies (blocks of 32 to
// 64 rows); false: the caller stores them otherwise.
template <int B>
__device__ __forceinline__ bool store_sym(uint8_t *dst, int prec, const double (&row)[B], int lane, double inv_s,
                                          int sym) {
  if constexpr (B >= 32) {
    if (sym) {
      if (lane < B) {
        switch (prec) {
          case P64: store_rows_sym<B, P64>(dst, row, lane, 1.0); break;
          case P32: store_rows_sym<B, P32>(dst, row, lane, inv_s); break;
          case PBF16: store_rows_sym<B, PBF16>(dst, row, lane, inv_s); break;
          default: store_rows_sym<B, P16>(dst, row, lane, inv_s); break;
        }
      }
      return true;
    }
  }
  return false;
}

template <int B>
__device__ __forceinline__ void store_block(uint8_t *dst, int prec, const double (&row)[B], int lane, double inv_s) {
  if (lane >= B) return;
  switch (prec) {
    case P64: store_rows<B, P64>(dst, row, lane, 1.0); break;
    case P32: store_rows<B, P32>(dst, row, lane, inv_s); break;
    case PBF16: store_rows<B, PBF16>(dst, row, lane, inv_s); break;
    default: store_rows<B, P16>(dst, row, lane, inv_s); break;
  }
}

// Band storage of one padded block: lane li writes E(d, li) = row[li + d]
// (times inv_s, rounded) for d = 0..w as entry d * B + li, zero where
// li + d >= B. The column index is a compile-time register index.
template <int P>
__device__ __forceinline__ void put_elem(uint8_t *p, double v) {
  if constexpr (P == P64) *(double *)p = v;
  else if constexpr (P == P32) *(uint32_t *)p = to_f32_bits(v);
  else *(uint16_t *)p = (uint16_t)to_bits<P>(v);
}

template <int B, int P>
__device__ __forceinline__ void store_band_rows(uint8_t *dst, const double (&row)[B], int lane, double inv_s, int w) {
  constexpr int BY = prec_bytes(P);
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int d = j - lane;
    if (d >= 0 && d <= w) put_elem<P>(dst + ((int64_t)d * B + lane) * BY, row[j] * inv_s);
  }
  for (int d = B - lane; d <= w; ++d) put_elem<P>(dst + ((int64_t)d * B + lane) * BY, 0.0);
}

template <int B>
__device__ __forceinline__ void store_band(uint8_t *dst, int prec, const double (&row)[B], int lane, double inv_s,
                                           int w) {
  if (lane >= B) return;
  switch (prec) {
    case P64: store_band_rows<B, P64>(dst, row, lane, 1.0, w); break;
    case P32: store_band_rows<B, P32>(dst, row, lane, inv_s, w); break;
    case PBF16: store_band_rows<B, PBF16>(dst, row, lane, inv_s, w); break;
    default: store_band_rows<B, P16>(dst, row, lane, inv_s, w); break;
  }
}

// Unit roundoff of each storage format, indexed by Prec.
__device__ __forceinline__ double unit_roundoff(int p) {
  return p == P64 ? 0x1p-53 : (p == P32 ? 0x1p-24 : (p == PBF16 ? 0x1p-8 : 0x1p-11));
}

__device__ __forceinline__ int ceil_log2(double v) {
  int e;
  const double m = frexp(v, &e);
  return (m == 0.5) ? e - 1 : e;
}

// One wave per diagonal block; lane i owns row i of the padded block
// diag(A_ii, I) (padded size B = b rounded up to a multiple of 16).
// Most entries in one row of the CSR (into *out, zeroed beforehand).
__global__ __launch_bounds__(256) void max_row_kernel(int64_t n, const int32_t *rp, int32_t *out) {
  int m = 0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = max(m, rp[i + 1] - rp[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

template <int B>
__global__ __launch_bounds__(256) void setup_kernel(SetupArgs a) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wid >= a.nblist) return;
  const int k = a.blist[wid];
  const int s = a.blk_row[k], e = a.blk_row[k + 1], b = e - s;
  const bool real = lane < b;

  double row[B];
#pragma unroll
  for (int j = 0; j < B; ++j) row[j] = (j == lane && !real) ? 1.0 : 0.0;

  // --- row quantities of the full CSR row (features) and the in-block row
  double d = 0.0, off_full = 0.0, off_in = 0.0, off2_in = 0.0, off2_out = 0.0;
  double tmax = -INFINITY, tmin = INFINITY, amax = -INFINITY, amin = INFINITY;
  if (real) {
    const int g = s + lane;
    for (int t = a.rp[g]; t < a.rp[g + 1]; ++t) {
      const int c = a.ci[t];
      const double v = a.val[t];
      const double av = fabs(v);
      const bool inb = c >= s && c < e;
      if (c == g) {
        d += v;
      } else {
        off_full += av;
        tmax = fmax(tmax, av);
        if (av > 0.0) tmin = fmin(tmin, av);
        if (inb) {
          off_in += av;
          off2_in += v * v;
        } else {
          off2_out += v * v;
        }
      }
      if (av > 0.0) {
        amax = fmax(amax, av);
        amin = fmin(amin, av);
      }
      if (inb) {
        const int jc = c - s;
#pragma unroll
        for (int j = 0; j < B; ++j)
          if (j == jc) row[j] += v;
      }
    }
  }

  // --- FP64 Gauss-Jordan sweep, no pivoting (pivots of an SPD block are the
  // positive Schur-complement diagonals). Pivot row k is broadcast from lane k.
  // The columns rotate left by one per step, so the pivot column is always
  // row[0] and the step loop needs no run-time register index (it stays a
  // loop: a fully unrolled B x B sweep spills and overflows the instruction
  // cache for B = 48, 64); after B steps the columns are back in place. Each
  // entry sees the same operations in the same order as the unrotated sweep.
  bool ok = true;
#pragma unroll 1
  for (int kk = 0; kk < B; ++kk) {
    double piv = bcast(row[0], kk);
    if (!(piv > 0.0)) {
      ok = false;
      piv = 1.0;
    }
    const double inv = 1.0 / piv;
    const double m = row[0] * inv;
    const bool isk = lane == kk;
#pragma unroll
    for (int j = 1; j < B; ++j) {
      const double pj = bcast(row[j], kk);
      row[j - 1] = isk ? pj * inv : fma(-m, pj, row[j]);
    }
    row[B - 1] = isk ? inv : -m;
  }
  if (!ok && lane == 0) {
    a.flags[k] = 1;
    atomicOr(a.any_bad, 1);
  }

  // --- features of H = A_ii^-1 (real rows and columns only)
  double hsum = 0.0, hmx = 0.0, hdiag = 0.0;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    if (real && j < b) {
      const double ah = fabs(row[j]);
      hsum += ah;
      hmx = fmax(hmx, ah);
    }
    if (j == lane) hdiag = row[j];
  }
  const double normH1 = wave_max(real ? hsum : 0.0);
  const double hmax = wave_max(hmx);
  const double hdmax = wave_max(real ? hdiag : -INFINITY);
  const double hdmin = wave_min(real ? hdiag : INFINITY);
  const double thr = ldexp(hmax, -24);
  double cnt = 0.0;
#pragma unroll
  for (int j = 0; j < B; ++j)
    if (real && j < b && fabs(row[j]) < thr) cnt += 1.0;
  const double nsmall = wave_sum(cnt);

  const double dom = real ? d / fmax(off_full, d / kDomCap) : INFINITY;
  const double dom_in = real ? d / fmax(off_in, d / kDomCap) : INFINITY;
  const bool hastau = isfinite(tmin) && tmax > 0.0;
  const double ltau = real ? (hastau ? log10(tmax / tmin) : 0.0) : 0.0;
  const double min_dom = wave_min(dom);
  const double sum_dom = wave_sum(real ? dom : 0.0);
  const double min_dom_in = wave_min(dom_in);
  const double s_off2_in = wave_sum(real ? off2_in : 0.0);
  const double s_off2_out = wave_sum(real ? off2_out : 0.0);
  const double s_d2 = wave_sum(real ? d * d : 0.0);
  const double max_lt = wave_max(real ? ltau : -INFINITY);
  const double sum_lt = wave_sum(ltau);
  const double mx_a = wave_max(real ? amax : -INFINITY);
  const double mn_a = wave_min(real ? amin : INFINITY);
  const double gl = wave_min(real ? d - off_in : INFINITY);
  const double gu = wave_max(real ? d + off_in : -INFINITY);
  const double dmax = wave_max(real ? d : -INFINITY);
  const double dmin = wave_min(real ? d : INFINITY);
  const double kappa1 = gu * normH1;

  if (a.feat && lane < 16) {
    double f;
    switch (lane) {
      case 0: f = b / 64.0; break;
      case 1: f = log10(min_dom); break;
      case 2: f = log10(sum_dom / b); break;
      case 3: f = log10(min_dom_in); break;
      case 4: f = sqrt(s_off2_in) / sqrt(s_d2); break;
      case 5: f = sqrt(s_off2_out) / sqrt(s_d2); break;
      case 6: f = max_lt; break;
      case 7: f = sum_lt / b; break;
      case 8: f = log10(mx_a / mn_a); break;
      case 9: f = gl / dmax; break;
      case 10: f = gu / dmax; break;
      case 11: f = log10(gu / fmax(gl, gu * kGershFloor)); break;
      case 12: f = log10(dmax / dmin); break;
      case 13: f = log10(kappa1); break;
      case 14: f = log10(hdmax / hdmin); break;
      default: f = nsmall / ((double)b * (double)b); break;
    }
    a.feat[(int64_t)k * 16 + lane] = (float)f;
  }

  // --- band widths: for each format the smallest w with
  // sum_{|i-j| > w} H_ij^2 <= tau^2 sum H_ij^2 (binary search; the dropped sum
  // shrinks as w grows, and every lane holds the same wave total)
  if (a.wband) {
    double t2 = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j)
      if (real && j < b) t2 = fma(row[j], row[j], t2);
    const double total = wave_sum(t2);
    for (int f = 0; f < 4; ++f) {
      const double u = a.band_rtol > 0.0 ? a.band_rtol : unit_roundoff(f);
      const double thr = u * u * total;
      int lo = 0, hi = b - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < B; ++j)
          if (real && j < b && abs(j - lane) > mid) t = fma(row[j], row[j], t);
        if (wave_sum(t) <= thr) hi = mid;
        else lo = mid + 1;
      }
      if (lane == 0) a.wband[(int64_t)k * 4 + f] = (uint8_t)lo;
    }
  }

  // --- precision of this block
  int tag;
  if (a.tag_mode == TAG_CONST) {
    tag = a.tag_const;
  } else if (a.tag_mode == TAG_ARRAY) {
    tag = a.tag_in[k];
  } else {
    tag = P64;
    if (kappa1 * 0x1p-24 <= a.theta) tag = P32;
    if (kappa1 * 0x1p-11 <= a.theta && min_dom * (1.0 + kDomSlack) >= a.d16) tag = P16;
  }
  if (a.tag_out && lane == 0) a.tag_out[k] = (uint8_t)tag;

  // --- scale, round, pack. The padding rows of diag(A_ii, I) are stored as
  // zeros: their outputs are never used, and 1/s of a scaled 16-bit block can
  // exceed the format (an infinity times a zero residual would be NaN)
  if (!real) {
#pragma unroll
    for (int j = 0; j < B; ++j) row[j] = 0.0;
  }
  if (a.off_hi) {
    if (a.w_hi) store_band<B>(a.base + a.off_hi[k], P64, row, lane, 1.0, a.w_hi[k]);
    else if (!store_sym<B>(a.base + a.off_hi[k], P64, row, lane, 1.0, a.sym))
      store_block<B>(a.base + a.off_hi[k], P64, row, lane, 1.0);
    if (lane == 0) a.scale_hi[k] = 1.0;
  }
  if (a.off_lo) {
    double sc = 1.0;
    if (tag == P16 || tag == PBF16) sc = ldexp(1.0, ceil_log2(hmax) - kScaleTopExp);
    if (!(a.off_hi && tag == P64)) {
      if (a.w_lo) store_band<B>(a.base + a.off_lo[k], tag, row, lane, 1.0 / sc, a.w_lo[k]);
      else if (!store_sym<B>(a.base + a.off_lo[k], tag, row, lane, 1.0 / sc, a.sym))
        store_block<B>(a.base + a.off_lo[k], tag, row, lane, 1.0 / sc);
    }
    if (lane == 0) a.scale_lo[k] = sc;
  }
}

static int launch_setup(const SetupArgs &base_args, const std::vector<std::vector<int32_t>> &cls,
                        int32_t *blist_dev, hipStream_t st) {
  int64_t off = 0;
  for (int c = 0; c < 4; ++c) {
    const int cnt = (int)cls[c].size();
    if (!cnt) continue;
    SetupArgs a = base_args;
    a.blist = blist_dev + off;
    a.nblist = cnt;
    dim3 grid((cnt + 3) / 4), blk(256);
    switch (c) {
      case 0: hipLaunchKernelGGL(setup_kernel<16>, grid, blk, 0, st, a); break;
      case 1: hipLaunchKernelGGL(setup_kernel<32>, grid, blk, 0, st, a); break;
      case 2: hipLaunchKernelGGL(setup_kernel<48>, grid, blk, 0, st, a); break;
      default: hipLaunchKernelGGL(setup_kernel<64>, grid, blk, 0, st, a); break;
    }
    MPB_HIP(hipGetLastError());
    off += cnt;
  }
  return BJAC_OK;
}

int launch_mlp_select(const float *feat, int32_t nb, const float *blob, uint8_t *tags, hipStream_t st);

struct Plan {
  int64_t n;
  int32_t nb;
  int32_t max_block;
  std::vector<int32_t> sizes;
  std::vector<uint8_t> bpad;       // padded size of each block (multiple of 16)
  int32_t uniform_b = 0;           // common padded size, 0 if sizes differ
  std::vector<int32_t> tiles;      // first block of each wave tile, + nb
  int64_t sum_b2 = 0;              // sum of padded B^2
  int64_t low_bound = 0, high_bytes = 0;
  bool temporal = false;
};

static int make_plan(const bjac_csr *A, const int32_t *bp, int32_t nb, const bjac_policy *pol, Plan &pl) {
  if (!A || !bp || !pol || nb < 1 || A->n < 1 || A->nnz < 0) return BJAC_EINVAL;
  if (bp[0] != 0 || bp[nb] != A->n || A->n >= (int64_t)1 << 31) return BJAC_EINVAL;
  if (pol->mode < BJAC_UNIFORM || pol->mode > BJAC_EXPLICIT) return BJAC_EINVAL;
  if (pol->temporal < BJAC_TEMPORAL_NONE || pol->temporal > BJAC_TEMPORAL_LH) return BJAC_EINVAL;
  if (pol->mode == BJAC_FIXED && (pol->low < BJAC_FP64 || pol->low > BJAC_FP16)) return BJAC_EINVAL;
  if (pol->mode == BJAC_EXPLICIT && !pol->explicit_tags) return BJAC_EINVAL;
  if (pol->mode == BJAC_LEARNED && !pol->mlp_blob) return BJAC_EINVAL;
  if (pol->storage < BJAC_STORE_FULL || pol->storage > BJAC_STORE_SYM) return BJAC_EINVAL;
  if (!(pol->band_rtol < 1.0)) return BJAC_EINVAL;  // NaN or >= 1
  pl.n = A->n;
  pl.nb = nb;
  pl.sizes.resize(nb);
  pl.max_block = 0;
  pl.temporal = pol->temporal != BJAC_TEMPORAL_NONE;
  int64_t lo_bytes_fixed = 0;
  pl.bpad.resize(nb);
  for (int32_t k = 0; k < nb; ++k) {
    const int32_t b = bp[k + 1] - bp[k];
    if (b < 1 || b > BJAC_MAX_BLOCK) return BJAC_EINVAL;
    pl.sizes[k] = b;
    pl.max_block = std::max(pl.max_block, b);
    pl.bpad[k] = (uint8_t)pad16(b);
  }
  // a remainder block smaller than all the others is padded to their common
  // size, so that workloads of equal blocks keep one storage shape
  bool uni = true;
  for (int32_t k = 1; k + 1 < nb; ++k) uni = uni && pl.bpad[k] == pl.bpad[0];
  if (uni && nb > 1 && pl.bpad[nb - 1] <= pl.bpad[0]) pl.bpad[nb - 1] = pl.bpad[0];
  pl.uniform_b = uni && (nb == 1 || pl.bpad[nb - 1] == pl.bpad[0]) ? pl.bpad[0] : 0;
  for (int32_t k = 0; k < nb; ++k) {
    const int64_t B = pl.bpad[k];
    pl.sum_b2 += B * B;
    if (pol->mode == BJAC_EXPLICIT) {
      const int t = pol->explicit_tags[k];
      if (t < 0 || t > 3) return BJAC_EINVAL;
      if (!(pl.temporal && t == P64)) lo_bytes_fixed += B * B * prec_bytes(t);
    }
  }
  // wave tiles: consecutive whole blocks, at most kWaveRows padded rows each
  pl.tiles.clear();
  int rows = kWaveRows;
  for (int32_t k = 0; k < nb; ++k) {
    const int B = pl.bpad[k];
    if (rows + B > kWaveRows) {
      pl.tiles.push_back(k);
      rows = 0;
    }
    rows += B;
  }
  pl.tiles.push_back(nb);
  pl.high_bytes = pl.temporal ? pl.sum_b2 * 8 : 0;
  switch (pol->mode) {
    case BJAC_UNIFORM: pl.low_bound = pl.temporal ? 0 : pl.sum_b2 * 8; break;
    case BJAC_FIXED:
      pl.low_bound = (pl.temporal && pol->low == BJAC_FP64) ? 0 : pl.sum_b2 * prec_bytes(pol->low);
      break;
    case BJAC_EXPLICIT: pl.low_bound = lo_bytes_fixed; break;
    default: pl.low_bound = pl.sum_b2 * (pl.temporal ? 4 : 8); break;
  }
  return BJAC_OK;
}

struct Layout {
  int32_t *blk_row, *tile_blk, *flags, *blist, *any_bad;
  int32_t *max_row;   // [1] most entries in one row of A
  uint8_t *bpad;
  int64_t *off_lo, *off_hi;
  double *scale_lo, *scale_hi;
  uint8_t *tag_lo, *tag_hi, *arena;
  uint8_t *wband, *w_lo, *w_hi;
  float *feat;
  size_t bytes;
};

static Layout carve(void *ws, const Plan &pl) {
  Carver c(ws);
  Layout L{};
  const int32_t nb = pl.nb;
  L.blk_row = c.take<int32_t>(nb + 1);
  L.tile_blk = c.take<int32_t>(pl.tiles.size());
  L.bpad = c.take<uint8_t>(nb);
  L.flags = c.take<int32_t>(nb);
  L.any_bad = c.take<int32_t>(1);
  L.max_row = c.take<int32_t>(1);
  L.blist = c.take<int32_t>(nb);
  L.off_lo = c.take<int64_t>(nb);
  L.off_hi = c.take<int64_t>(nb);
  L.scale_lo = c.take<double>(nb);
  L.scale_hi = c.take<double>(nb);
  L.tag_lo = c.take<uint8_t>(nb);
  L.tag_hi = c.take<uint8_t>(nb);
  L.feat = c.take<float>((size_t)nb * 16);
  L.wband = c.take<uint8_t>((size_t)nb * 4);
  L.w_lo = c.take<uint8_t>(nb);
  L.w_hi = c.take<uint8_t>(nb);
  L.arena = c.take<uint8_t>((size_t)(pl.high_bytes + pl.low_bound) + 256);
  L.bytes = c.used;
  return L;
}

}  // namespace mpb

using namespace mpb;

extern "C" int bjac_setup_query(const bjac_csr *A, const int32_t *block_ptr, int32_t nb,
                                const bjac_policy *policy, size_t *workspace_bytes) {
  if (!workspace_bytes) return BJAC_EINVAL;
  Plan pl;
  int rc = make_plan(A, block_ptr, nb, policy, pl);
  if (rc) return rc;
  *workspace_bytes = carve(nullptr, pl).bytes;
  return BJAC_OK;
}

extern "C" int bjac_setup(const bjac_csr *A, const int32_t *block_ptr, int32_t nb, const bjac_policy *policy,
                          void *workspace, size_t workspace_bytes, void *stream, bjac_handle **out) {
  if (!out || !workspace || !A || !A->row_ptr || !A->col_idx || !A->val) return BJAC_EINVAL;
  *out = nullptr;
  Plan pl;
  int rc = make_plan(A, block_ptr, nb, policy, pl);
  if (rc) return rc;
  Layout L = carve(workspace, pl);
  if (L.bytes > workspace_bytes) return BJAC_ENOMEM;
  hipStream_t st = (hipStream_t)stream;

  auto h = new bjac_handle();
  h->n = pl.n;
  h->nb = nb;
  h->max_block = pl.max_block;
  h->ntiles = (int32_t)pl.tiles.size() - 1;
  h->policy = *policy;
  h->policy.explicit_tags = nullptr;
  h->stream = st;
  h->ws = (uint8_t *)workspace;
  h->ws_bytes = workspace_bytes;
  h->blk_row = L.blk_row;
  h->tile_blk = L.tile_blk;
  h->bpad = L.bpad;
  h->uniform_b = pl.uniform_b;
  h->h_bpad = pl.bpad;
  h->off_lo = L.off_lo;
  h->off_hi = pl.temporal ? L.off_hi : nullptr;
  h->scale_lo = L.scale_lo;
  h->scale_hi = pl.temporal ? L.scale_hi : nullptr;
  h->tag_lo = L.tag_lo;
  h->tag_hi = pl.temporal ? L.tag_hi : nullptr;
  h->feat = L.feat;
  h->flags = L.flags;
  h->h_blk_row.assign(block_ptr, block_ptr + nb + 1);

  auto fail = [&](int code) {
    (void)hipStreamSynchronize(st);
    delete h;
    return code;
  };

  // size classes of padded blocks
  std::vector<std::vector<int32_t>> cls(4);
  for (int32_t k = 0; k < nb; ++k) cls[pl.bpad[k] / 16 - 1].push_back(k);
  std::vector<int32_t> blist;
  blist.reserve(nb);
  for (auto &c : cls) blist.insert(blist.end(), c.begin(), c.end());

  if (hipMemcpyAsync(L.blk_row, block_ptr, sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(L.tile_blk, pl.tiles.data(), sizeof(int32_t) * pl.tiles.size(), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(L.bpad, pl.bpad.data(), nb, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(L.blist, blist.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st) ||
      hipMemsetAsync(L.flags, 0, sizeof(int32_t) * nb, st) || hipMemsetAsync(L.any_bad, 0, sizeof(int32_t), st) ||
      hipMemsetAsync(L.max_row, 0, sizeof(int32_t), st))
    return fail(BJAC_EHIP);
  {
    const int g = (int)std::min<int64_t>(1024, (A->n + 255) / 256);
    hipLaunchKernelGGL(max_row_kernel, dim3(std::max(g, 1)), dim3(256), 0, st, (int64_t)A->n, A->row_ptr, L.max_row);
  }

  SetupArgs a{};
  a.rp = A->row_ptr;
  a.ci = A->col_idx;
  a.val = A->val;
  a.blk_row = L.blk_row;
  a.theta = policy->theta > 0 ? policy->theta : 1e-2;
  a.d16 = policy->d16 > 0 ? policy->d16 : 1.0;
  a.flags = L.flags;
  a.any_bad = L.any_bad;
  a.base = (uint8_t *)workspace;
  a.feat = L.feat;

  // precision map (and, for band storage, the widths) on the host
  const bool band = policy->storage == BJAC_STORE_BAND;
  const bool sym = policy->storage == BJAC_STORE_SYM;
  a.band_rtol = policy->band_rtol;
  std::vector<uint8_t> tags(nb, 0), wb;
  const int mode = policy->mode;
  const bool data_map = mode == BJAC_RULE || mode == BJAC_LEARNED;
  if (data_map || band) {
    SetupArgs p1 = a;
    p1.tag_mode = TAG_RULE;
    p1.tag_out = (mode == BJAC_RULE) ? L.tag_lo : nullptr;
    p1.wband = band ? L.wband : nullptr;
    if ((rc = launch_setup(p1, cls, L.blist, st))) return fail(rc);
    if (mode == BJAC_LEARNED && (rc = launch_mlp_select(L.feat, nb, policy->mlp_blob, L.tag_lo, st)))
      return fail(rc);
    if (data_map && hipMemcpyAsync(tags.data(), L.tag_lo, nb, hipMemcpyDeviceToHost, st)) return fail(BJAC_EHIP);
    if (band) {
      wb.resize((size_t)nb * 4);
      if (hipMemcpyAsync(wb.data(), L.wband, wb.size(), hipMemcpyDeviceToHost, st)) return fail(BJAC_EHIP);
    }
    if (hipStreamSynchronize(st)) return fail(BJAC_EHIP);
  }
  if (mode == BJAC_FIXED) {
    std::fill(tags.begin(), tags.end(), (uint8_t)policy->low);
  } else if (mode == BJAC_EXPLICIT) {
    std::memcpy(tags.data(), policy->explicit_tags, nb);
  }
  // stored bytes of block k in format p: B^2 entries, w + 1 diagonals of B,
  // or the upper strips of a symmetric block (B (B + 16) / 2 entries)
  auto width = [&](int32_t k, int p) -> int { return band ? wb[(size_t)k * 4 + p] : 0; };
  auto blk_elems = [&](int B) -> int64_t { return sym ? (int64_t)sym_elems(B) : (int64_t)B * B; };
  auto blk_bytes = [&](int32_t k, int p) -> int64_t {
    const int64_t B = pl.bpad[k];
    return (band ? B * (width(k, p) + 1) : blk_elems((int)B)) * prec_bytes(p);
  };
  // offsets: the FP64 map first (temporal), then the low map; in temporal
  // handles FP64 blocks of the low map alias the FP64 map
  std::vector<int64_t> off_lo(nb), off_hi(nb, 0);
  const int64_t arena0 = L.arena - (uint8_t *)workspace;
  int64_t o = arena0;
  int64_t hi_bytes = 0;
  if (pl.temporal) {
    for (int32_t k = 0; k < nb; ++k) {
      off_hi[k] = o;
      o += blk_bytes(k, P64);
    }
    hi_bytes = o - arena0;
  }
  int64_t lo_bytes = 0, lo_all = 0;
  for (int32_t k = 0; k < nb; ++k) {
    const int64_t bb = blk_bytes(k, tags[k]);
    lo_all += bb;
    if (pl.temporal && tags[k] == P64) {
      off_lo[k] = off_hi[k];
    } else {
      off_lo[k] = o;
      o += bb;
      lo_bytes += bb;
    }
    h->hist[tags[k]]++;
  }
  if (o - arena0 > pl.high_bytes + pl.low_bound) return fail(BJAC_EINVAL);
  h->low_bytes = pl.temporal ? lo_all : lo_bytes;
  h->high_bytes = hi_bytes;
  if (hipMemcpyAsync(L.off_lo, off_lo.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(L.tag_lo, tags.data(), nb, hipMemcpyHostToDevice, st))
    return fail(BJAC_EHIP);
  if (band) {
    h->h_w_lo.resize(nb);
    h->h_w_hi.resize(nb);
    for (int32_t k = 0; k < nb; ++k) {
      h->h_w_lo[k] = (uint8_t)width(k, tags[k]);
      h->h_w_hi[k] = (uint8_t)width(k, P64);
    }
    if (hipMemcpyAsync(L.w_lo, h->h_w_lo.data(), nb, hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(L.w_hi, h->h_w_hi.data(), nb, hipMemcpyHostToDevice, st))
      return fail(BJAC_EHIP);
    h->storage = BJAC_STORE_BAND;
    h->w_lo = L.w_lo;
    h->w_hi = pl.temporal ? L.w_hi : nullptr;
  }
  if (sym) h->storage = BJAC_STORE_SYM;
  if (pl.temporal) {
    std::vector<uint8_t> t64(nb, 0);
    if (hipMemcpyAsync(L.off_hi, off_hi.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(L.tag_hi, t64.data(), nb, hipMemcpyHostToDevice, st) || hipStreamSynchronize(st))
      return fail(BJAC_EHIP);
  }
  if (band && hipStreamSynchronize(st)) return fail(BJAC_EHIP);

  SetupArgs p2 = a;
  p2.tag_mode = TAG_ARRAY;
  p2.tag_in = L.tag_lo;
  p2.off_lo = L.off_lo;
  p2.scale_lo = L.scale_lo;
  p2.off_hi = pl.temporal ? L.off_hi : nullptr;
  p2.scale_hi = L.scale_hi;
  p2.w_lo = band ? L.w_lo : nullptr;
  p2.w_hi = (band && pl.temporal) ? L.w_hi : nullptr;
  p2.sym = sym ? 1 : 0;
  if ((rc = launch_setup(p2, cls, L.blist, st))) return fail(rc);
  int32_t bad = 0, max_row = 0;
  if (hipMemcpyAsync(&bad, L.any_bad, sizeof(int32_t), hipMemcpyDeviceToHost, st) ||
      hipMemcpyAsync(&max_row, L.max_row, sizeof(int32_t), hipMemcpyDeviceToHost, st) || hipStreamSynchronize(st))
    return fail(BJAC_EHIP);
  h->max_row_nnz = max_row;
  if (bad) return fail(BJAC_ENOTSPD);
  h->h_tag_lo = tags;
  h->uprec_lo = tags[0];
  for (int32_t k = 1; k < nb; ++k)
    if (tags[k] != tags[0]) h->uprec_lo = -1;
  bool rows_uniform = pl.uniform_b > 0;
  for (int32_t k = 0; k + 1 < nb && rows_uniform; ++k) rows_uniform = pl.sizes[k] == pl.uniform_b;
  h->rows_uniform = rows_uniform;
  if (rows_uniform && h->uprec_lo >= 0 && !band) {
    const int64_t stride = blk_elems(pl.uniform_b) * prec_bytes(h->uprec_lo);
    bool contig = true;
    for (int32_t k = 0; k < nb && contig; ++k) contig = off_lo[k] == off_lo[0] + k * stride;
    h->fast_lo = contig;
    h->lo_off0 = off_lo[0];
  }
  if (rows_uniform && pl.temporal && !band) {
    const int64_t stride = blk_elems(pl.uniform_b) * 8;
    bool contig = true;
    for (int32_t k = 0; k < nb && contig; ++k) contig = off_hi[k] == off_hi[0] + k * stride;
    h->fast_hi = contig;
    h->hi_off0 = off_hi[0];
  }
  h->h_off_lo = off_lo;
  h->h_off_hi = off_hi;
  *out = h;
  return BJAC_OK;
}

extern "C" void bjac_destroy(bjac_handle *h) {
  if (!h) return;
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
}

extern "C" int bjac_get_info(const bjac_handle *h, bjac_info *info) {
  if (!h || !info) return BJAC_EINVAL;
  info->n = h->n;
  info->nb = h->nb;
  info->max_block = h->max_block;
  for (int i = 0; i < 4; ++i) info->blocks_per_prec[i] = h->hist[i];
  info->low_bytes = h->low_bytes;
  info->high_bytes = h->high_bytes;
  info->temporal = h->policy.temporal;
  info->mode = h->policy.mode;
  info->ntiles = h->ntiles;
  info->reserved = 0;
  return BJAC_OK;
}

extern "C" int bjac_get_tags(const bjac_handle *h, uint8_t *tags) {
  if (!h || !tags) return BJAC_EINVAL;
  std::memcpy(tags, h->h_tag_lo.data(), h->nb);
  return BJAC_OK;
}

extern "C" int bjac_get_features(const bjac_handle *h, float *features) {
  if (!h || !features || h->kind != 0) return BJAC_EINVAL;
  MPB_HIP(hipMemcpyAsync(features, h->feat, sizeof(float) * 16 * (size_t)h->nb, hipMemcpyDeviceToHost, h->stream));
  MPB_HIP(hipStreamSynchronize(h->stream));
  return BJAC_OK;
}

static double decode(const uint8_t *p, int prec) {
  switch (prec) {
    case P64: { double v; std::memcpy(&v, p, 8); return v; }
    case P32: { float v; std::memcpy(&v, p, 4); return v; }
    case PBF16: {
      uint16_t u; std::memcpy(&u, p, 2);
      uint32_t w = (uint32_t)u << 16; float v; std::memcpy(&v, &w, 4); return v;
    }
    default: {
      uint16_t u; std::memcpy(&u, p, 2);
      const int ex = (u >> 10) & 31, man = u & 1023;
      double v = ex == 0 ? std::ldexp((double)man, -24)
                 : ex == 31 ? (man ? NAN : INFINITY) : std::ldexp(1024.0 + man, ex - 25);
      return (u & 0x8000) ? -v : v;
    }
  }
}

extern "C" int bjac_get_block(const bjac_handle *h, int32_t which, int32_t block, double *out, double *scale) {
  if (!h || !out || block < 0 || block >= h->nb || h->kind != 0) return BJAC_EINVAL;
  if (which == 1 && !h->off_hi) return BJAC_EINVAL;
  const int b = h->h_blk_row[block + 1] - h->h_blk_row[block];
  const int B = h->h_bpad[block];
  const int prec = which == 1 ? P64 : h->h_tag_lo[block];
  const int64_t off = which == 1 ? h->h_off_hi[block] : h->h_off_lo[block];
  const int BY = prec_bytes(prec), V = 16 / BY;
  const bool band = h->storage == BJAC_STORE_BAND;
  const bool sym = h->storage == BJAC_STORE_SYM;
  const int w = band ? (which == 1 ? h->h_w_hi[block] : h->h_w_lo[block]) : 0;
  std::vector<uint8_t> raw((size_t)(sym ? sym_elems(B) : B * (band ? w + 1 : B)) * BY);
  double sc = 1.0;
  MPB_HIP(hipMemcpyAsync(raw.data(), h->ws + off, raw.size(), hipMemcpyDeviceToHost, h->stream));
  MPB_HIP(hipMemcpyAsync(&sc, (which == 1 ? h->scale_hi : h->scale_lo) + block, sizeof(double),
                         hipMemcpyDeviceToHost, h->stream));
  MPB_HIP(hipStreamSynchronize(h->stream));
  for (int i = 0; i < b; ++i) {
    for (int j = 0; j < b; ++j) {
      if (sym) {
        // row tile I keeps columns 16 I .. B-1 as strip I; an entry left of
        // its row tile's strip is the mirror of a stored one
        const bool lower = (j / 16) < (i / 16);
        const int ri = lower ? j : i, rj = lower ? i : j;
        const int I = ri / 16;
        const int64_t e = sym_strip_off(B, I) + layout_elem(B - 16 * I, V, ri % 16, rj - 16 * I);
        out[(size_t)i * b + j] = decode(raw.data() + e * BY, prec);
      } else if (!band) {
        out[(size_t)i * b + j] = decode(raw.data() + layout_elem(B, V, i, j) * BY, prec);
      } else {
        const int d = std::abs(i - j);
        out[(size_t)i * b + j] = d > w ? 0.0 : decode(raw.data() + ((size_t)d * B + std::min(i, j)) * BY, prec);
      }
    }
  }
  if (scale) *scale = sc;
  return BJAC_OK;
}

extern "C" int bjac_get_band(const bjac_handle *h, int32_t which, uint8_t *w) {
  if (!h || !w || h->kind != 0 || h->storage != BJAC_STORE_BAND) return BJAC_EINVAL;
  if (which == 1 && !h->w_hi) return BJAC_EINVAL;
  if (which != 0 && which != 1) return BJAC_EINVAL;
  const std::vector<uint8_t> &src = which == 1 ? h->h_w_hi : h->h_w_lo;
  std::memcpy(w, src.data(), h->nb);
  return BJAC_OK;
}
