// Device helpers shared by the mpbjac kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpb {

constexpr int kWave = 64;

// ------------------------------------------------------------ wave reductions
// Butterfly over the 64 lanes; every lane ends with the same association order
// per lane, and the order is fixed, so results are run-to-run deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  return v;
}

// Value of lane `src` (wave-uniform) broadcast to all lanes.
__device__ __forceinline__ double bcast(double v, int src) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// ------------------------------------------------- storage formats and rounding
enum Prec : int { P64 = 0, P32 = 1, PBF16 = 2, P16 = 3 };

__host__ __device__ constexpr int prec_bytes(int p) { return p == P64 ? 8 : (p == P32 ? 4 : 2); }

// Round an FP64 value to the nearest value of a binary format with PB
// significand bits (hidden bit included), minimum normal exponent EMIN and
// EB exponent bits: ties to even, gradual underflow, overflow to infinity,
// NaN kept quiet. Works on the integer image of the double, so it does not
// depend on the FP32 denormal mode of the hardware and never double-rounds.
template <int PB, int EMIN, int EB>
__device__ __forceinline__ uint32_t round_f64_bits(double d) {
  constexpr int MB = PB - 1;
  constexpr int BIAS = (1 << (EB - 1)) - 1;
  constexpr uint32_t INF = ((1u << EB) - 1u) << MB;
  const uint64_t u = (uint64_t)__double_as_longlong(d);
  const uint32_t sign = (uint32_t)(u >> 63) << (EB + MB);
  const int ex = (int)((u >> 52) & 0x7ff);
  const uint64_t mant = u & 0xFFFFFFFFFFFFFull;
  if (ex == 0x7ff) return sign | INF | (mant ? (1u << (MB - 1)) : 0u);
  if (ex == 0) return sign;                              // zero or FP64 subnormal
  const int E = ex - 1023;
  const uint64_t M = (1ull << 52) | mant;                 // 53-bit significand
  const int shift = 53 - PB + (E < EMIN ? (EMIN - E) : 0);
  if (shift >= 54) return sign;                           // below half the smallest subnormal
  uint64_t q = M >> shift;
  const uint64_t rem = M & ((1ull << shift) - 1ull);
  const uint64_t half = 1ull << (shift - 1);
  if (rem > half || (rem == half && (q & 1ull))) ++q;
  if (E < EMIN) return sign | (uint32_t)q;                // subnormal (carry gives min normal)
  int Eo = E;
  if (q == (1ull << PB)) { q >>= 1; ++Eo; }
  if (Eo + BIAS >= (1 << EB) - 1) return sign | INF;
  return sign | ((uint32_t)(Eo + BIAS) << MB) | (uint32_t)(q & ((1ull << MB) - 1ull));
}
__device__ __forceinline__ uint32_t to_f32_bits(double d) { return round_f64_bits<24, -126, 8>(d); }
__device__ __forceinline__ uint32_t to_bf16_bits(double d) { return round_f64_bits<8, -126, 8>(d); }
__device__ __forceinline__ uint32_t to_f16_bits(double d) { return round_f64_bits<11, -14, 5>(d); }

template <int P>
__device__ __forceinline__ uint32_t to_bits(double d) {
  if constexpr (P == P32) return to_f32_bits(d);
  else if constexpr (P == PBF16) return to_bf16_bits(d);
  else return to_f16_bits(d);
}

// Decoding of stored values to FP32 (exact for all three formats).
__device__ __forceinline__ float f16_bits(uint16_t u) { return (float)__builtin_bit_cast(_Float16, u); }
__device__ __forceinline__ float f16_lo(uint32_t w) { return f16_bits((uint16_t)(w & 0xffffu)); }
__device__ __forceinline__ float f16_hi(uint32_t w) { return f16_bits((uint16_t)(w >> 16)); }
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// -------------------------------------------------------- block storage layout
// A block of padded size B (multiple of 16, <= 64) is stored as B/16 row tiles
// of 16 rows. Inside a row tile the columns form B/4 k-steps of 4 columns.
// Lane slot l = (row % 16) + 16 * (col % 4) owns, for every k-step, one value;
// a lane's values for V consecutive k-steps (V = 16 bytes / element size) are
// contiguous, so one 16-byte load per lane fetches V k-steps, and the 64 lanes
// of a wave read one contiguous 1 KiB segment per load. This is the operand
// layout of the 16x16x4 matrix-core instructions (A operand: lane l holds
// A[l % 16][l / 16]) and serves the vector apply and the matrix-core batched
// apply alike. The last group of k-steps may be shorter than V.
__host__ __device__ constexpr int64_t layout_group_base(int B, int V, int mt, int g) {
  return (int64_t)mt * 64 * (B / 4) + (int64_t)g * 64 * V;
}
__host__ __device__ constexpr int layout_vg(int B, int V, int g) {
  return (B / 4 - g * V) < V ? (B / 4 - g * V) : V;
}
__host__ __device__ constexpr int64_t layout_elem(int B, int V, int i, int j) {
  // element (i, j) of the padded block
  return layout_group_base(B, V, i / 16, (j / 4) / V) +
         (int64_t)((i % 16) + 16 * (j % 4)) * layout_vg(B, V, (j / 4) / V) + (j / 4) % V;
}

__host__ __device__ constexpr int pad16(int b) { return (b + 15) & ~15; }

}  // namespace mpb
