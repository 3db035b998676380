// common.cuh -- device helpers shared by the libsmash kernels.
#pragma once

#include "internal.h"

namespace smash {

constexpr int WAVE = 64;

// BF16 operands of the 16x16x32 matrix-core step (eight per lane) and the
// FP32 accumulator tile.  Conversions round to nearest even.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  return __builtin_bit_cast(unsigned short, (__bf16)x);
}

// Exclusive block scan of one int64 per thread (blockDim a multiple of 64).
// lds must hold blockDim/64 + 1 entries.  Ends with a barrier, so lds may be
// reused right after.
__device__ inline int64_t block_excl_scan_i64(int64_t v, int64_t *total, int64_t *lds) {
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  const int nw = blockDim.x / WAVE;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int64_t y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if (lane == WAVE - 1) lds[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int w = 0; w < nw; w++) {
      int64_t t = lds[w];
      lds[w] = s;
      s += t;
    }
    lds[nw] = s;
  }
  __syncthreads();
  int64_t r = x - v + lds[wid];
  *total = lds[nw];
  __syncthreads();
  return r;
}
// the same for a compile-time count NW of wavefronts per workgroup
template <int NW>
__device__ inline int64_t block_excl_scan_i64(int64_t v, int64_t *total, int64_t *lds) {
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int64_t y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if (lane == WAVE - 1) lds[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int w = 0; w < NW; w++) {
      int64_t t = lds[w];
      lds[w] = s;
      s += t;
    }
    lds[NW] = s;
  }
  __syncthreads();
  int64_t r = x - v + lds[wid];
  *total = lds[NW];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ kernels
// kappa(x, y) in FP64.  "x = y" means every coordinate equal (eq. (2.1):
// the diagonal value d_x is then returned for the singular kernels).
// Natural logarithm of a positive double for the kernel log|x - y|, by
// argument reduction and the atanh series: x = 2^e m with m in
// [sqrt(1/2), sqrt(2)) and log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),
// s = (m - 1) / (m + 1), |s| < 0.172, so the terms through s^21 leave a
// truncation below 3e-17 relative; e ln 2 is added in double-double
// (ln 2 = LN2_HI + LN2_LO, the nearest double and the rest).  A few units in
// the last place, at about a third of the library routine's instructions;
// zero, infinity and NaN go to the library routine.
constexpr double LN2_HI = 0.6931471805599453;     // nearest double to ln 2
constexpr double LN2_LO = 2.319046813846299558e-17;  // ln 2 - LN2_HI
__device__ __forceinline__ double log_pos(double x) {
  if (!(x > 0.0 && x < __builtin_huge_val())) return log(x);
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1), exact
  int e = __builtin_amdgcn_frexp_exp(x);
  if (m < 0.70710678118654752440) {
    m += m;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);  // m - 1 is exact
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double s2 = s + s;
  const double lm = fma(s2 * z, p, s2);  // 2 atanh(s)
  const double de = (double)e;
  const double hi = de * LN2_HI;
  const double he = fma(de, LN2_HI, -hi);  // the product's rounding error, exactly
  return hi + (lm + (he + de * LN2_LO));
}

// 1/sqrt(x) for x > 0 in FP64: the hardware reciprocal-square-root estimate
// refined by two Newton-Raphson steps for x^(-1/2),
// y <- y + (y / 2) (1 - x y^2), the residual from one fused multiply-add;
// within a unit or two in the last place, at about a third of the
// instructions of a square root followed by a division.  x outside
// (2^-900, 2^900) (subnormal, zero, infinite, NaN) goes to those.
__device__ __forceinline__ double inv_sqrt_pos(double x) {
  if (!(x > 0x1p-900 && x < 0x1p+900)) return 1.0 / sqrt(x);
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; it++) {
    const double t = x * y;
    const double e = fma(-t, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Laplace double layer (Sec. 6.4, eq. (6.9)) in Nystrom form, dim 2:
// grad_y Phi(x, y) . m_y with Phi = -log|x - y| / (2 pi), i.e.
// -((y - x) . m_y) / (2 pi |x - y|^2); ay = the column point's data
// (m_1, m_2, .), ax = the row point's (., ., diagonal value).
__device__ __forceinline__ double double_layer_f64(const double *x, const double *y, double r2,
                                                   bool same, const double *ax,
                                                   const double *ay) {
  if (same) return ax[2];
  const double proj = (y[0] - x[0]) * ay[0] + (y[1] - x[1]) * ay[1];
  return -proj / (2.0 * M_PI * r2);
}
__device__ __forceinline__ float double_layer_f32(const double *x, const double *y, float r2,
                                                  bool same, const double *ax,
                                                  const double *ay) {
  if (same) return (float)ax[2];
  const float proj = (float)(y[0] - x[0]) * (float)ay[0] + (float)(y[1] - x[1]) * (float)ay[1];
  return -proj / ((float)(2.0 * M_PI) * r2);
}

// ax, ay: the row and column points' data (the double-layer kernel only)
__device__ inline double kernel_f64(int kid, const double *x, const double *y, int d,
                                    double diag, const double *ax = nullptr,
                                    const double *ay = nullptr) {
  double r2 = 0.0;
  bool same = true;
  for (int t = 0; t < d; t++) {
    double df = x[t] - y[t];
    same = same && (x[t] == y[t]);
    r2 += df * df;
  }
  if (kid == SMASH_KERNEL_EXP_R) return exp(-sqrt(r2));
  if (kid == SMASH_KERNEL_DOUBLE_LAYER) return double_layer_f64(x, y, r2, same, ax, ay);
  if (same) return diag;
  if (kid == SMASH_KERNEL_INV_R) return inv_sqrt_pos(r2);
  if (kid == SMASH_KERNEL_LOG_R) return 0.5 * log_pos(r2);
  return 1.0 / (x[0] - y[0]);
}

// FP32 evaluation: coordinate differences are formed in FP64 (points may be
// closer than FP32 resolution), the rest in FP32.
__device__ inline float kernel_f32(int kid, const double *x, const double *y, int d,
                                   float diag, const double *ax = nullptr,
                                   const double *ay = nullptr) {
  float r2 = 0.0f;
  bool same = true;
  float dx0 = 0.0f;
  for (int t = 0; t < d; t++) {
    double df = x[t] - y[t];
    same = same && (x[t] == y[t]);
    float f = (float)df;
    if (t == 0) dx0 = f;
    r2 += f * f;
  }
  if (kid == SMASH_KERNEL_EXP_R) return __expf(-sqrtf(r2));
  if (kid == SMASH_KERNEL_DOUBLE_LAYER) return double_layer_f32(x, y, r2, same, ax, ay);
  if (same) return diag;
  if (kid == SMASH_KERNEL_INV_R) return rsqrtf(r2);
  if (kid == SMASH_KERNEL_LOG_R) return 0.5f * __logf(r2);
  return 1.0f / dx0;
}

// The same two evaluations with the kernel and the dimension fixed at
// compile time (identical operations in the same order, so identical
// results); the block evaluation instantiates them per kernel and dim.
template <int KID, int D>
__device__ __forceinline__ double kernel_f64_t(const double *x, const double *y, double diag,
                                               const double *ax = nullptr,
                                               const double *ay = nullptr) {
  double r2 = 0.0;
  bool same = true;
#pragma unroll
  for (int t = 0; t < D; t++) {
    double df = x[t] - y[t];
    same = same && (x[t] == y[t]);
    r2 += df * df;
  }
  if (KID == SMASH_KERNEL_EXP_R) return exp(-sqrt(r2));
  if (KID == SMASH_KERNEL_DOUBLE_LAYER) return double_layer_f64(x, y, r2, same, ax, ay);
  if (same) return diag;
  if (KID == SMASH_KERNEL_INV_R) return inv_sqrt_pos(r2);
  if (KID == SMASH_KERNEL_LOG_R) return 0.5 * log_pos(r2);
  return 1.0 / (x[0] - y[0]);
}

template <int KID, int D>
__device__ __forceinline__ float kernel_f32_t(const double *x, const double *y, float diag,
                                              const double *ax = nullptr,
                                              const double *ay = nullptr) {
  float r2 = 0.0f;
  bool same = true;
  float dx0 = 0.0f;
#pragma unroll
  for (int t = 0; t < D; t++) {
    double df = x[t] - y[t];
    same = same && (x[t] == y[t]);
    float f = (float)df;
    if (t == 0) dx0 = f;
    r2 += f * f;
  }
  if (KID == SMASH_KERNEL_EXP_R) return __expf(-sqrtf(r2));
  if (KID == SMASH_KERNEL_DOUBLE_LAYER) return double_layer_f32(x, y, r2, same, ax, ay);
  if (same) return diag;
  if (KID == SMASH_KERNEL_INV_R) return rsqrtf(r2);
  if (KID == SMASH_KERNEL_LOG_R) return 0.5f * __logf(r2);
  return 1.0f / dx0;
}

// Def. 2.1, eq. (2.3) on boxes: delta_i + delta_j <= tau |c_i - c_j| with c
// the box centre and delta half its diagonal, decided exactly without a
// square root: e = tau^2 D^2 - delta_i^2 - delta_j^2 >= 0 and
// 4 delta_i^2 delta_j^2 <= e^2.  The library is compiled without FP
// contraction, so this is the same rounding sequence on every run.
__device__ inline bool well_separated(const double *lo, const double *hi, int i, int j, int d,
                                      double tau) {
  double di2 = 0.0, dj2 = 0.0, D2 = 0.0;
  for (int t = 0; t < d; t++) {
    double wi = hi[3 * i + t] - lo[3 * i + t];
    double wj = hi[3 * j + t] - lo[3 * j + t];
    di2 += wi * wi;
    dj2 += wj * wj;
    double ci = 0.5 * (lo[3 * i + t] + hi[3 * i + t]);
    double cj = 0.5 * (lo[3 * j + t] + hi[3 * j + t]);
    double dc = ci - cj;
    D2 += dc * dc;
  }
  di2 = 0.25 * di2;
  dj2 = 0.25 * dj2;
  double e = tau * tau * D2 - di2 - dj2;
  if (e < 0.0) return false;
  return 4.0 * di2 * dj2 <= e * e;
}

}  // namespace smash
