// Linear kernels (Alg. 1 CallLinear): kick and drift, streaming over slots
// (SoA) or records (AoS), and the FP64 conservation reductions.
#include "sph_device.h"

namespace sph {
namespace {

constexpr int kThreads = 256;
constexpr int kReduceBlocks = 1024;
constexpr int kReduceVals = 8;

// Kick v and u with the FP32 rates, drift x in FP64 with the kicked v, wrap.
// Returns whether the particle's cell changed.
__device__ __forceinline__ bool kick_drift_one(double x[3], float v[3], float& u,
                                               const float a[3], float du, float dtk, double dtd,
                                               int n_c) {
  bool moved = false;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v[c] = __builtin_fmaf(a[c], dtk, v[c]);
    double xn = __builtin_fma((double)v[c], dtd, x[c]);
    xn = wrap01(xn);
    moved |= cell_axis(wrap01(x[c]), n_c) != cell_axis(xn, n_c);
    x[c] = xn;
  }
  u = __builtin_fmaf(du, dtk, u);
  return moved;
}

__device__ __forceinline__ void count_moved(bool moved, int32_t* counter) {
  uint64_t b = __ballot(moved);
  if (counter && (threadIdx.x & 63) == 0 && b) atomicAdd(counter, (int)__popcll(b));
}

struct KickSoa {
  double* x[3];
  float* v[3];
  float* u;
  const float* a[3];
  const float* du;
};

__global__ __launch_bounds__(kThreads) void k_kick_drift(KickSoa s, int n, int n_c, float dtk,
                                                          double dtd, int32_t* moved) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  bool mv = false;
  if (k < n) {
    double x[3];
    float v[3], a[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] = s.x[c][k];
      v[c] = s.v[c][k];
      a[c] = s.a[c][k];
    }
    float u = s.u[k];
    mv = kick_drift_one(x, v, u, a, s.du[k], dtk, dtd, n_c);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s.x[c][k] = x[c];
      s.v[c][k] = v[c];
    }
    s.u[k] = u;
  }
  count_moved(mv, moved);
}

__global__ __launch_bounds__(kThreads) void k_kick_drift_aos(char* __restrict__ aos, AosLayout L,
                                                              int n, int n_c, float dtk,
                                                              double dtd, int32_t* moved) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  bool mv = false;
  if (k < n) {
    char* rec = aos + (size_t)k * L.stride;
    double* xp = reinterpret_cast<double*>(rec + L.off[SPH_A_X]);
    double x[3];
    float v[3], a[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] = wrap01(xp[c]);
      v[c] = rec_load32(rec, L.off[SPH_A_V], L.dt[SPH_A_V], c);
      a[c] = rec_load32(rec, L.off[SPH_A_A], L.dt[SPH_A_A], c);
    }
    float u = rec_load32(rec, L.off[SPH_A_U], L.dt[SPH_A_U]);
    const float du = rec_load32(rec, L.off[SPH_A_DU], L.dt[SPH_A_DU]);
    mv = kick_drift_one(x, v, u, a, du, dtk, dtd, n_c);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xp[c] = x[c];
      rec_store32(rec, L.off[SPH_A_V], L.dt[SPH_A_V], v[c], c);
    }
    rec_store32(rec, L.off[SPH_A_U], L.dt[SPH_A_U], u);
  }
  count_moved(mv, moved);
}

struct RedSoa {
  const void* m;
  int mhu_dt;
  float lm;
  const void* v[3];
  int vel_dt;
  const float* a[3];
  const float* du;
  const int32_t* nngb;
  const int32_t* nforce;
};

__global__ __launch_bounds__(kThreads) void k_reduce_partial(RedSoa s, int n,
                                                              double* __restrict__ part) {
  __shared__ double lds[kThreads / 64][kReduceVals];
  double acc[kReduceVals];
#pragma unroll
  for (int q = 0; q < kReduceVals; ++q) acc[q] = 0.0;
  for (int k = blockIdx.x * kThreads + threadIdx.x; k < n; k += gridDim.x * kThreads) {
    const double m = s.m ? (double)load_q(s.m, s.mhu_dt, k, s.lm) : 1.0;
    double va = 0.0, an = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a = s.a[c][k];
      const double v = load_q(s.v[c], s.vel_dt, k, 1.0f);
      acc[c] += m * a;
      va += v * a;
      an += a * a;
    }
    const double du = s.du[k];
    acc[3] += m * (va + du);
    acc[4] += m * sqrt(an);
    acc[5] += m * (fabs(va) + fabs(du));
    acc[6] += s.nngb ? (double)s.nngb[k] : 0.0;
    acc[7] += s.nforce ? (double)s.nforce[k] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kReduceVals; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    acc[q] = v;
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < kReduceVals; ++q) lds[threadIdx.x >> 6][q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x < kReduceVals) {
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += lds[w][threadIdx.x];
    part[blockIdx.x * kReduceVals + threadIdx.x] = t;
  }
}

// Sum the per-block partials of each value in a fixed order: thread t adds
// partials t, t + 256, ..., then a fixed shuffle/LDS tree combines threads.
__global__ __launch_bounds__(kThreads) void k_reduce_final(const double* __restrict__ part, int nb,
                                                            double* __restrict__ out) {
  __shared__ double lds[kThreads / 64];
  for (int q = 0; q < kReduceVals; ++q) {
    double t = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) t += part[b * kReduceVals + q];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) r += lds[w];
      out[q] = r;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_kick_drift(const sph_soa& soa, const CellsDev& c, double dtk, double dtd,
                             int32_t* moved, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  KickSoa k;
  for (int a = 0; a < 3; ++a) {
    k.x[a] = static_cast<double*>(soa.f[SPH_S_X_X + a]);
    k.v[a] = static_cast<float*>(soa.f[SPH_S_V_X + a]);
    k.a[a] = static_cast<const float*>(soa.f[SPH_S_A_X + a]);
  }
  k.u = static_cast<float*>(soa.f[SPH_S_UK]);
  k.du = static_cast<const float*>(soa.f[SPH_S_DU]);
  k_kick_drift<<<(c.n + kThreads - 1) / kThreads, kThreads, 0, s>>>(k, c.n, c.n_c, (float)dtk,
                                                                     dtd, moved);
  return hipGetLastError();
}

hipError_t launch_kick_drift_aos(void* aos, const AosLayout& L, int n, int n_c, double dtk,
                                 double dtd, int32_t* moved, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_kick_drift_aos<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(
      static_cast<char*>(aos), L, n, n_c, (float)dtk, dtd, moved);
  return hipGetLastError();
}

size_t reduce_workspace_bytes(int n) {
  (void)n;
  return sizeof(double) * kReduceBlocks * kReduceVals;
}

hipError_t launch_reduce(const sph_soa& soa, const Prec& p, int n, double* out, void* ws,
                         hipStream_t s) {
  RedSoa r;
  r.m = soa.f[SPH_S_M];
  r.mhu_dt = p.mhu;
  r.lm = p.load_m;
  for (int a = 0; a < 3; ++a) {
    r.v[a] = soa.f[SPH_S_VQ_X + a];
    r.a[a] = static_cast<const float*>(soa.f[SPH_S_A_X + a]);
  }
  r.vel_dt = p.vel;
  r.du = static_cast<const float*>(soa.f[SPH_S_DU]);
  r.nngb = static_cast<const int32_t*>(soa.f[SPH_S_NNGB]);
  r.nforce = static_cast<const int32_t*>(soa.f[SPH_S_NFORCE]);
  double* part = static_cast<double*>(ws);
  k_reduce_partial<<<kReduceBlocks, kThreads, 0, s>>>(r, n, part);
  k_reduce_final<<<1, kThreads, 0, s>>>(part, kReduceBlocks, out);
  return hipGetLastError();
}

}  // namespace sph
