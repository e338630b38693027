// Smoothing lengths adapted to the local density (Sec. 2.1: h follows the
// density so that the neighbour number stays about constant), from
// h = eta (m / rho)^(1/3). The density loop gathers with h_i, so rho_i is a
// function of particle i's own h and every particle solves its own
//   f(h) = h - eta (m / rho(h))^(1/3) = 0
// by Newton steps, f'(h) = 1 + (h_t / (3 rho)) drho/dh with
// h_t = eta (m / rho(h))^(1/3) and drho/dh the density loop's RHO_DH; a step
// that f' <= 0 would make is replaced by h_t, every new h is limited to
// [h/2, 2h] and to h_max (the largest h whose support fits a cell), and a
// particle is done after the first step with |h_new - h| < tol h that the
// h_max limit did not cut. The host loop (sph_smoothing_length) alternates
// the density loop over the cells that still hold active particles with
// launch_hiter_update.
//
// Workspace: active flags [n] (1: still iterating), per-block counts of the
// particles left active, and their sum.
#include "sph_device.h"

namespace sph {
namespace {

constexpr int kThreads = 256;

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

struct HiterWs {
  uint8_t* active;
  int32_t* partial;   // [blocks]
  int32_t* left;      // [1]
};

HiterWs carve(void* ws, int n) {
  char* p = static_cast<char*>(ws);
  HiterWs w;
  w.active = reinterpret_cast<uint8_t*>(p);
  p += al256((size_t)(n > 0 ? n : 1));
  w.partial = reinterpret_cast<int32_t*>(p);
  p += al256(sizeof(int32_t) * (size_t)cdiv(n > 0 ? n : 1, kThreads));
  w.left = reinterpret_cast<int32_t*>(p);
  return w;
}

__global__ __launch_bounds__(kThreads) void k_hiter_init(float* __restrict__ H, int n,
                                                          float lh, float sh, float h_max,
                                                          uint8_t* __restrict__ active) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= n) return;
  const float h = H[k] * lh;
  if (h > h_max) H[k] = h_max * sh;
  active[k] = 1;
}

__global__ __launch_bounds__(kThreads) void k_hiter_update(float* __restrict__ H,
                                                            const float* __restrict__ rho,
                                                            const float* __restrict__ rho_dh,
                                                            const void* __restrict__ m, int mdt,
                                                            float lm, float lh, float sh, int n,
                                                            float eta, float tol, float h_max,
                                                            uint8_t* __restrict__ active,
                                                            int32_t* __restrict__ partial) {
  __shared__ int wcount[kThreads / 64];
  const int k = blockIdx.x * kThreads + threadIdx.x;
  bool left = false;
  if (k < n && active[k]) {
    const float h = H[k] * lh;
    const float r = rho[k];
    const float ht = eta * cbrtf(load_q(m, mdt, k, lm) / r);
    const float f = h - ht;
    const float fp = 1.0f + ht / (3.0f * r) * rho_dh[k];
    float hn = fp > 0.0f ? h - f / fp : ht;
    hn = fminf(fmaxf(hn, 0.5f * h), 2.0f * h);
    const bool capped = hn > h_max;
    if (capped) hn = h_max;
    const bool done = !capped && fabsf(hn - h) < tol * h;
    H[k] = hn * sh;
    active[k] = done ? 0 : 1;
    left = !done;
  }
  const uint64_t b = __ballot(left);
  if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kThreads / 64; ++w) s += wcount[w];
    partial[blockIdx.x] = s;
  }
}

// sum of the per-block counts, one workgroup, fixed order
__global__ __launch_bounds__(kThreads) void k_sum_partials(const int32_t* __restrict__ partial,
                                                            int nb, int32_t* __restrict__ out) {
  __shared__ int red[kThreads];
  int s = 0;
  for (int i = threadIdx.x; i < nb; i += kThreads) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// largest h of each cell, from the SoA values: one wave per cell, so a
// crowded cell's slots are read 64 at a time
__global__ __launch_bounds__(kThreads) void k_cell_hmax(const int32_t* __restrict__ start, int C,
                                                         int n, const void* __restrict__ H,
                                                         int hdt, float lh,
                                                         float* __restrict__ hmax) {
  const int c = blockIdx.x * (kThreads / 64) + (int)(threadIdx.x >> 6);
  if (c >= C) return;                       // whole waves leave together
  const int lane = threadIdx.x & 63;
  const int a = min(max(start[c], 0), n), b = min(max(start[c + 1], a), n);
  float m = 0.0f;
  for (int k = a + lane; k < b; k += 64) m = fmaxf(m, load_q(H, hdt, k, lh));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) hmax[c] = m;
}

// h of slot k into the H field of record perm[k]
__global__ __launch_bounds__(kThreads) void k_write_h(const void* __restrict__ H, int hdt,
                                                       float lh, const int32_t* __restrict__ perm,
                                                       int n, char* __restrict__ aos,
                                                       AosLayout L) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= n) return;
  const int r = min(max(perm[k], 0), n - 1);
  rec_store32(aos + (size_t)r * L.stride, L.off[SPH_A_H], L.dt[SPH_A_H], load_q(H, hdt, k, lh));
}

}  // namespace

size_t hiter_workspace_bytes(int n) {
  const int nn = n > 0 ? n : 1;
  return al256((size_t)nn) + al256(sizeof(int32_t) * (size_t)cdiv(nn, kThreads)) + 256;
}

hipError_t launch_hiter_init(const sph_soa& soa, const Prec& p, int n, float h_max, void* ws,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  HiterWs w = carve(ws, n);
  k_hiter_init<<<cdiv(n, kThreads), kThreads, 0, s>>>(static_cast<float*>(soa.f[SPH_S_H]), n,
                                                       p.load_h, p.store_h, h_max, w.active);
  return hipGetLastError();
}

hipError_t launch_hiter_update(const sph_soa& soa, const Prec& p, int n, float eta, float tol,
                               float h_max, void* ws, hipStream_t s) {
  HiterWs w = carve(ws, n);
  const int nb = cdiv(n > 0 ? n : 1, kThreads);
  if (n > 0)
    k_hiter_update<<<nb, kThreads, 0, s>>>(
        static_cast<float*>(soa.f[SPH_S_H]), static_cast<const float*>(soa.f[SPH_S_RHO]),
        static_cast<const float*>(soa.f[SPH_S_RHO_DH]), soa.f[SPH_S_M], p.mhu, p.load_m,
        p.load_h, p.store_h, n, eta, tol, h_max, w.active, w.partial);
  else
    k_sum_partials<<<1, kThreads, 0, s>>>(w.partial, 0, w.left);
  if (n > 0) k_sum_partials<<<1, kThreads, 0, s>>>(w.partial, nb, w.left);
  return hipGetLastError();
}

const uint8_t* hiter_active(void* ws, int n) { return carve(ws, n).active; }
const int32_t* hiter_left(void* ws, int n) { return carve(ws, n).left; }

hipError_t launch_cell_hmax(const sph_soa& soa, const Prec& p, const CellsDev& c, float* hmax,
                            hipStream_t s) {
  const int C = c.n_c * c.n_c * c.n_c;
  k_cell_hmax<<<cdiv(C, kThreads / 64), kThreads, 0, s>>>(c.start, C, c.n, soa.f[SPH_S_H], p.mhu,
                                                           p.load_h, hmax);
  return hipGetLastError();
}

hipError_t launch_write_h(const sph_soa& soa, const Prec& p, const CellsDev& c, void* aos,
                          const AosLayout& L, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  k_write_h<<<cdiv(c.n, kThreads), kThreads, 0, s>>>(soa.f[SPH_S_H], p.mhu, p.load_h, c.perm,
                                                      c.n, static_cast<char*>(aos), L);
  return hipGetLastError();
}

}  // namespace sph
