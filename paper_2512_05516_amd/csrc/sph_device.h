// Device-side helpers shared by the HIP kernels of libsphmi: typed field
// access, storage quantisers, cell arithmetic, the FP32 support test and the
// cubic-spline kernel. Host code never includes this file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sph_internal.h"

namespace sph {

// ---------------------------------------------------------------------------
// Storage formats (Table 2 rows 32 and 16, plus bfloat16). Conversions use
// the hardware RNE instructions: v_cvt_f32_f64, v_cvt_f16_f32,
// v_cvt_pk_bf16_f32; widening is exact.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_f16_bits(float v) {
  return __builtin_bit_cast(uint16_t, (_Float16)v);
}
__device__ __forceinline__ float f16_bits_to_f32(uint16_t b) {
  return (float)__builtin_bit_cast(_Float16, b);
}
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float v) {
  return __builtin_bit_cast(uint16_t, (__bf16)v);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

// truncate_mantissa storage of T bits (9 <= T <= 32; Table 2): the code of a
// value is the top T bits of its IEEE single (T > 16) or half (T <= 16)
// pattern, i.e. the mantissa cut toward zero; codes are packed into a
// little-endian bitstream of 32-bit words, value k at bits [kT, kT + T).
__device__ __forceinline__ uint32_t trunc_code(float q, int T) {
  if (T > 16) return __float_as_uint(q) >> (32 - T);
  return (uint32_t)f32_to_f16_bits(q) >> (16 - T);
}
__device__ __forceinline__ float trunc_load(const void* p, int T, int64_t k) {
  const uint32_t* w = static_cast<const uint32_t*>(p);
  const uint64_t b = (uint64_t)k * (uint64_t)T;
  const uint64_t i = b >> 5;
  const uint64_t v = (uint64_t)w[i] | ((uint64_t)w[i + 1] << 32);
  const uint32_t code = (uint32_t)(v >> (b & 31)) & (T == 32 ? 0xffffffffu : (1u << T) - 1u);
  if (T > 16) return __uint_as_float(code << (32 - T));
  return f16_bits_to_f32((uint16_t)(code << (16 - T)));
}

// Read element k of an array stored in `dt`, widened to FP32, times `scale`
// (an exact power of two, 1 when unscaled).
__device__ __forceinline__ float load_q(const void* p, int dt, int64_t k, float scale) {
  float v;
  if (dt >= DT_TRUNC) v = trunc_load(p, dt - DT_TRUNC, k);
  else if (dt == DT_F32) v = static_cast<const float*>(p)[k];
  else if (dt == DT_F16) v = f16_bits_to_f32(static_cast<const uint16_t*>(p)[k]);
  else v = bf16_bits_to_f32(static_cast<const uint16_t*>(p)[k]);
  return v * scale;
}

// Store FP64 value v as RNE(RNE32(v) * scale) in format dt.
__device__ __forceinline__ void store_q(void* p, int dt, int64_t k, double v, float scale) {
  float q = (float)v * scale;
  if (dt == DT_F32) static_cast<float*>(p)[k] = q;
  else if (dt == DT_F16) static_cast<uint16_t*>(p)[k] = f32_to_f16_bits(q);
  else static_cast<uint16_t*>(p)[k] = f32_to_bf16_bits(q);
}

// Store an FP32 value (already in registers) in format dt.
__device__ __forceinline__ void store_q32(void* p, int dt, int64_t k, float v, float scale) {
  float q = v * scale;
  if (dt == DT_F32) static_cast<float*>(p)[k] = q;
  else if (dt == DT_F16) static_cast<uint16_t*>(p)[k] = f32_to_f16_bits(q);
  else static_cast<uint16_t*>(p)[k] = f32_to_bf16_bits(q);
}

// AoS record fields: FP32 or FP64 floating elements, read as double.
__device__ __forceinline__ double rec_load(const char* rec, uint32_t off, int dt, int c = 0) {
  if (dt == DT_F64) return reinterpret_cast<const double*>(rec + off)[c];
  return (double)reinterpret_cast<const float*>(rec + off)[c];
}
__device__ __forceinline__ float rec_load32(const char* rec, uint32_t off, int dt, int c = 0) {
  if (dt == DT_F64) return (float)reinterpret_cast<const double*>(rec + off)[c];
  return reinterpret_cast<const float*>(rec + off)[c];
}
__device__ __forceinline__ void rec_store32(char* rec, uint32_t off, int dt, float v, int c = 0) {
  if (off == kAbsent) return;
  if (dt == DT_F64) reinterpret_cast<double*>(rec + off)[c] = (double)v;
  else reinterpret_cast<float*>(rec + off)[c] = v;
}
__device__ __forceinline__ void rec_store_i32(char* rec, uint32_t off, int32_t v) {
  if (off == kAbsent) return;
  *reinterpret_cast<int32_t*>(rec + off) = v;
}

// ---------------------------------------------------------------------------
// Cells of the periodic unit box
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wrap01(double x) { return x - floor(x); }

// per-axis cell index of a wrapped coordinate; NaN maps to 0 (flagged
// separately by the binning kernel)
__device__ __forceinline__ int cell_axis(double xw, int n_c) {
  double t = floor(xw * (double)n_c);
  int c = (t == t) ? (int)fmin(fmax(t, 0.0), (double)(n_c - 1)) : 0;
  return c;
}

__device__ __forceinline__ void cell_coords(int c, int n_c, int& cx, int& cy, int& cz) {
  cx = c % n_c;
  cy = (c / n_c) % n_c;
  cz = c / (n_c * n_c);
}

// Cells in brick order: bricks of 4 x 4 x 4 cells (thinner at the upper box
// edge when n_c is not a multiple of 4) taken x-fastest, then y, then z, the
// cells of a brick x-fastest. Maps an index j in [0, n_c^3) to a cell id and
// is a bijection. Launches that visit cells in this order keep the
// neighbourhood of the cells in flight small enough for an XCD's L2; the
// plain id order has each cell's z-neighbours n_c^2 cells apart.
constexpr int kBrick = 4;
__device__ __forceinline__ int brick_cell(int j, int n_c) {
  const int nb = (n_c + kBrick - 1) / kBrick;
  const int last = n_c - kBrick * (nb - 1);          // side of the last brick of an axis
  const int layer = kBrick * n_c * n_c;              // cells of a full z-layer of bricks
  const int bz = min(j / layer, nb - 1);
  int r = j - bz * layer;
  const int tz = bz == nb - 1 ? last : kBrick;
  const int row = tz * kBrick * n_c;                 // cells of a full row of bricks
  const int by = min(r / row, nb - 1);
  r -= by * row;
  const int ty = by == nb - 1 ? last : kBrick;
  const int col = tz * ty * kBrick;                  // cells of a full brick
  const int bx = min(r / col, nb - 1);
  r -= bx * col;
  const int tx = bx == nb - 1 ? last : kBrick;
  const int lx = r % tx, ly = (r / tx) % ty, lz = r / (tx * ty);
  return (kBrick * bx + lx) + n_c * ((kBrick * by + ly) + n_c * (kBrick * bz + lz));
}

// FP32 offset of a wrapped coordinate from its cell origin c / n_c: the
// FP64 difference rounded once.
__device__ __forceinline__ float cell_offset(double xw, int c_axis, int n_c) {
  return (float)(xw - (double)c_axis / (double)n_c);
}

// FP32 offset of a wrapped coordinate from its anchor, the FP64 difference
// rounded once: SPH_ANCHOR_CORNER, the cell corner c / n_c (a = 0);
// SPH_ANCHOR_SUB(b), the centre (c 2^b + a + 1/2) / (n_c 2^b) of its
// sub-cell a = floor(xw n_c 2^b) - c 2^b, clamped to [0, 2^b - 1].
__device__ __forceinline__ float anchor_offset(double xw, int c_axis, int n_c, int anchor,
                                               int& a) {
  if (anchor == SPH_ANCHOR_CORNER) {
    a = 0;
    return cell_offset(xw, c_axis, n_c);
  }
  const int R = 1 << (anchor - 1);
  const double t = floor(xw * (double)(n_c * R));
  a = (t == t) ? (int)fmin(fmax(t - (double)c_axis * R, 0.0), (double)(R - 1)) : 0;
  const double o = ((double)c_axis * R + a + 0.5) / ((double)n_c * R);
  return (float)(xw - o);
}

// ---------------------------------------------------------------------------
// FP32 support test. With xr = off_j + shift (one FP32 add, shift in
// {-s, 0, s}) and d = off_i - xr, the squared distance is
// fma(dz, dz, fma(dy, dy, dx * dx)); the decision is r2 < (gamma_k h)^2
// with H = gamma_k * h and H * H rounded in FP32. The arithmetic is spelled
// out with contraction off so every build takes the same decisions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float shifted(float off, float shift) {
#pragma clang fp contract(off)
  return off + shift;
}

__device__ __forceinline__ float dist2(float xi, float yi, float zi, float xr, float yr,
                                       float zr, float& dx, float& dy, float& dz) {
#pragma clang fp contract(off)
  dx = xi - xr;
  dy = yi - yr;
  dz = zi - zr;
  float xx = dx * dx;
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, xx));
}

__device__ __forceinline__ float support2(float gamma_k32, float h) {
#pragma clang fp contract(off)
  float H = gamma_k32 * h;
  return H * H;
}

// ---------------------------------------------------------------------------
// Cubic-spline M4 kernel (Sec. 2.1) on the unit support, FP32:
// w(u) = 8/pi (1 - 6u^2 + 6u^3) for u < 1/2, 16/pi (1-u)^3 for u < 1.
// ---------------------------------------------------------------------------
constexpr float kC8 = 2.5464790894703255f;    // 8/pi
constexpr float kC16 = 5.092958178940651f;    // 16/pi
constexpr float kC48 = 15.278874536821952f;   // 48/pi
constexpr float kFourPiThird = 4.1887902047863905f;

__device__ __forceinline__ void kernel_w_dw(float u, float& w, float& dw) {
  float t = 1.0f - u;
  float wi = kC8 * (1.0f + u * u * (6.0f * u - 6.0f));
  float dwi = kC8 * u * (18.0f * u - 12.0f);
  float wo = kC16 * t * t * t;
  float dwo = -kC48 * t * t;
  bool inner = u < 0.5f;
  w = inner ? wi : wo;
  dw = inner ? dwi : dwo;
}

__device__ __forceinline__ float kernel_dw(float u) {
  float t = 1.0f - u;
  float dwi = kC8 * u * (18.0f * u - 12.0f);
  float dwo = -kC48 * t * t;
  float d = u < 0.5f ? dwi : dwo;
  return u < 1.0f ? d : 0.0f;
}

// Wendland C2 on the unit support, FP32: w(u) = 21/(2 pi) (1-u)^4 (1+4u),
// w'(u) = -210/pi u (1-u)^3, both zero for u >= 1.
constexpr float kCW = 3.3422538049298023f;    // 21/(2 pi)
constexpr float kCWd = 66.84507609859604f;    // 210/pi

__device__ __forceinline__ void wendland_w_dw(float u, float& w, float& dw) {
  const float t = fmaxf(1.0f - u, 0.0f);
  const float t3 = t * t * t;
  w = kCW * (t3 * t) * (1.0f + 4.0f * u);
  dw = -kCWd * u * t3;
}

__device__ __forceinline__ float wendland_dw(float u) {
  const float t = fmaxf(1.0f - u, 0.0f);
  return -kCWd * u * (t * t * t);
}

// Kernel shape as a compile-time tag: the loops branch once per batch on
// the launch's (uniform) kernel choice and run a specialised body.
template <int KS>
struct KernelShape {
  static constexpr int value = KS;
  __device__ __forceinline__ static void w_dw(float u, float& w, float& dw) {
    if (KS == SPH_KERNEL_WENDLAND_C2) wendland_w_dw(u, w, dw);
    else kernel_w_dw(u, w, dw);
  }
  __device__ __forceinline__ static float dw(float u) {
    return KS == SPH_KERNEL_WENDLAND_C2 ? wendland_dw(u) : kernel_dw(u);
  }
};

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// wave64 helpers
__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << __lane_id()) - 1ull;
}

}  // namespace sph
