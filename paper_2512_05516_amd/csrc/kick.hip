// Linear kernels (Alg. 1 CallLinear): kick and drift, streaming over slots
// (SoA) or records (AoS), and the FP64 conservation reductions.
#include <mutex>

#include "sph_device.h"

namespace sph {
namespace {

constexpr int kThreads = 256;
constexpr int kReduceBlocks = 1024;
constexpr int kReduceVals = 8;

// The cell along one axis of a wrapped coordinate and, at depth sub_bits,
// the sub-cell inside it (the binning's definitions), as one integer.
__device__ __forceinline__ int cell_sub_axis(double xw, int n_c, int sub_bits) {
  const int c = cell_axis(xw, n_c);
  if (sub_bits == 0) return c;
  const int R = 1 << sub_bits;
  const double t = floor(xw * (double)(n_c * R));
  const int sa = (t == t) ? (int)fmin(fmax(t - (double)c * R, 0.0), (double)(R - 1)) : 0;
  return c * R + sa;
}

// Kick v and u with the FP32 rates, drift x in FP64 with the kicked v, wrap.
// Returns whether the particle's cell (or sub-cell at depth sub_bits)
// changed.
__device__ __forceinline__ bool kick_drift_one(double x[3], float v[3], float& u,
                                               const float a[3], float du, float dtk, double dtd,
                                               int n_c, int sub_bits) {
  bool moved = false;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v[c] = __builtin_fmaf(a[c], dtk, v[c]);
    double xn = __builtin_fma((double)v[c], dtd, x[c]);
    xn = wrap01(xn);
    moved |= cell_sub_axis(wrap01(x[c]), n_c, sub_bits) != cell_sub_axis(xn, n_c, sub_bits);
    x[c] = xn;
  }
  u = __builtin_fmaf(du, dtk, u);
  return moved;
}

// Adds the block's count of moved particles to *counter: one atomic per
// block that has any.
__device__ __forceinline__ void count_moved(bool moved, int32_t* counter) {
  __shared__ int wsum[kThreads / 64];
  const uint64_t b = __ballot(moved);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = (int)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0 && counter) {
    int t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += wsum[w];
    if (t) atomicAdd(counter, t);
  }
}

struct KickSoa {
  double* x[3];
  float* v[3];
  float* u;
  const float* a[3];
  const float* du;
};

// One slot per thread. Every field is streamed once (read, then written in
// place), so loads and stores are non-temporal: the lines go through the
// caches without displacing data that is reused (measured on 4M slots
// beyond the Infinity Cache: 4.1 -> 5.3 TB/s at 96 B per slot).
__global__ __launch_bounds__(kThreads) void k_kick_drift(KickSoa s, int n, int n_c, int sub_bits,
                                                          float dtk, double dtd, int32_t* moved) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  bool mv = false;
  if (k < n) {
    double x[3];
    float v[3], a[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] = __builtin_nontemporal_load(s.x[c] + k);
      v[c] = __builtin_nontemporal_load(s.v[c] + k);
      a[c] = __builtin_nontemporal_load(s.a[c] + k);
    }
    float u = __builtin_nontemporal_load(s.u + k);
    const float du = __builtin_nontemporal_load(s.du + k);
    mv = kick_drift_one(x, v, u, a, du, dtk, dtd, n_c, sub_bits);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      __builtin_nontemporal_store(x[c], s.x[c] + k);
      __builtin_nontemporal_store(v[c], s.v[c] + k);
    }
    __builtin_nontemporal_store(u, s.u + k);
  }
  count_moved(mv, moved);
}

__global__ __launch_bounds__(kThreads) void k_kick_drift_aos(char* __restrict__ aos, AosLayout L,
                                                              int n, int n_c, int sub_bits,
                                                              float dtk, double dtd,
                                                              int32_t* moved) {
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
    mv = kick_drift_one(x, v, u, a, du, dtk, dtd, n_c, sub_bits);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xp[c] = x[c];
      rec_store32(rec, L.off[SPH_A_V], L.dt[SPH_A_V], v[c], c);
    }
    rec_store32(rec, L.off[SPH_A_U], L.dt[SPH_A_U], u);
  }
  count_moved(mv, moved);
}

// Inputs of the reductions at slot k: the SoA arrays (m and v in their
// storage formats), or the AoS records through the cell list (record
// perm[k]), in the same slot order, so FP32 storage and FP32 records give
// the same sums bit for bit.
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

  __device__ __forceinline__ double mass(int k) const {
    return m ? (double)load_q(m, mhu_dt, k, lm) : 1.0;
  }
  __device__ __forceinline__ double vel(int k, int c) const {
    return load_q(v[c], vel_dt, k, 1.0f);
  }
  __device__ __forceinline__ double acc(int k, int c) const { return a[c][k]; }
  __device__ __forceinline__ double dudt(int k) const { return du[k]; }
  __device__ __forceinline__ double ngb(int k) const { return nngb ? (double)nngb[k] : 0.0; }
  __device__ __forceinline__ double nfrc(int k) const { return nforce ? (double)nforce[k] : 0.0; }
};

struct RedAos {
  const char* aos;
  AosLayout L;
  const int32_t* perm;
  int n;

  __device__ __forceinline__ const char* rec(int k) const {
    return aos + (size_t)min(max(perm[k], 0), n - 1) * L.stride;
  }
  __device__ __forceinline__ double mass(int k) const {
    return L.off[SPH_A_M] != kAbsent ? (double)rec_load32(rec(k), L.off[SPH_A_M], L.dt[SPH_A_M])
                                     : 1.0;
  }
  __device__ __forceinline__ double vel(int k, int c) const {
    return rec_load32(rec(k), L.off[SPH_A_V], L.dt[SPH_A_V], c);
  }
  __device__ __forceinline__ double acc(int k, int c) const {
    return rec_load32(rec(k), L.off[SPH_A_A], L.dt[SPH_A_A], c);
  }
  __device__ __forceinline__ double dudt(int k) const {
    return rec_load32(rec(k), L.off[SPH_A_DU], L.dt[SPH_A_DU]);
  }
  __device__ __forceinline__ double count(int k, int f) const {
    return L.off[f] != kAbsent ? (double)*reinterpret_cast<const int32_t*>(rec(k) + L.off[f])
                               : 0.0;
  }
  __device__ __forceinline__ double ngb(int k) const { return count(k, SPH_A_NNGB); }
  __device__ __forceinline__ double nfrc(int k) const { return count(k, SPH_A_NFORCE); }
};

template <class R>
__global__ __launch_bounds__(kThreads) void k_reduce_partial(R s, int n,
                                                              double* __restrict__ part) {
  __shared__ double lds[kThreads / 64][kReduceVals];
  double acc[kReduceVals];
#pragma unroll
  for (int q = 0; q < kReduceVals; ++q) acc[q] = 0.0;
  for (int k = blockIdx.x * kThreads + threadIdx.x; k < n; k += gridDim.x * kThreads) {
    const double m = s.mass(k);
    double va = 0.0, an = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a = s.acc(k, c);
      const double v = s.vel(k, c);
      acc[c] += m * a;
      va += v * a;
      an += a * a;
    }
    const double du = s.dudt(k);
    acc[3] += m * (va + du);
    acc[4] += m * sqrt(an);
    acc[5] += m * (fabs(va) + fabs(du));
    acc[6] += s.ngb(k);
    acc[7] += s.nfrc(k);
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

// --- leapfrog support: predicted v, u; time step and conserved totals -----

struct PredIn {
  const float* v[3];      // kick view V (half-step values)
  const float* u;         // kick view UK
  void* vq[3];            // force view VQ (stored format)
  void* uq;               // U (stored format)
  int vel_dt, mhu_dt;
  float store_u;
  const int32_t* perm;
  const char* aos;
  AosLayout L;
};

// v and u predicted to the end of the step with the last rates (record
// fields A, DU of the slot's record), stored in the force/density formats.
__global__ __launch_bounds__(kThreads) void k_predict(PredIn s, int n, float dth) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= n) return;
  const char* rec = s.aos + (size_t)min(max(s.perm[k], 0), n - 1) * s.L.stride;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float a = rec_load32(rec, s.L.off[SPH_A_A], s.L.dt[SPH_A_A], c);
    store_q32(s.vq[c], s.vel_dt, k, __builtin_fmaf(a, dth, s.v[c][k]), 1.0f);
  }
  const float du = rec_load32(rec, s.L.off[SPH_A_DU], s.L.dt[SPH_A_DU]);
  store_q32(s.uq, s.mhu_dt, k, __builtin_fmaf(du, dth, s.u[k]), s.store_u);
}

struct TotIn {
  const void* m;
  const void* h;
  int mhu_dt;
  float lm, lh;
  const float* v[3];
  const float* u;
  const float* vsig;
  double gk, cfl;
};

// Per-block partials: sums of m v (3), m |v|^2 / 2, m u, m, the count of
// slots with vsig > 0 (slot 7) and the minimum CFL step (slot 6).
__global__ __launch_bounds__(kThreads) void k_totals_partial(TotIn s, int n,
                                                             double* __restrict__ part) {
  __shared__ double lds[kThreads / 64][kReduceVals];
  double acc[kReduceVals];
#pragma unroll
  for (int q = 0; q < kReduceVals; ++q) acc[q] = 0.0;
  acc[6] = __builtin_inf();
  for (int k = blockIdx.x * kThreads + threadIdx.x; k < n; k += gridDim.x * kThreads) {
    const double m = (double)load_q(s.m, s.mhu_dt, k, s.lm);
    double v2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = s.v[c][k];
      acc[c] += m * v;
      v2 += v * v;
    }
    acc[3] += 0.5 * m * v2;
    acc[4] += m * (double)s.u[k];
    acc[5] += m;
    const double vs = s.vsig[k];
    if (vs > 0.0) {
      const double h = (double)load_q(s.h, s.mhu_dt, k, s.lh);
      acc[6] = fmin(acc[6], s.cfl * (s.gk * h) / vs);
      acc[7] += 1.0;
    }
  }
#pragma unroll
  for (int q = 0; q < kReduceVals; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) {
      const double w = __shfl_xor(v, o);
      v = (q == 6) ? fmin(v, w) : v + w;
    }
    acc[q] = v;
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < kReduceVals; ++q) lds[threadIdx.x >> 6][q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x < kReduceVals) {
    const int q = threadIdx.x;
    double t = (q == 6) ? __builtin_inf() : 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t = (q == 6) ? fmin(t, lds[w][q]) : t + lds[w][q];
    part[blockIdx.x * kReduceVals + q] = t;
  }
}

__global__ __launch_bounds__(kThreads) void k_totals_final(const double* __restrict__ part, int nb,
                                                           double* __restrict__ out) {
  __shared__ double lds[kThreads / 64];
  for (int q = 0; q < kReduceVals; ++q) {
    const bool mn = q == 6;
    double t = mn ? __builtin_inf() : 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) {
      const double x = part[b * kReduceVals + q];
      t = mn ? fmin(t, x) : t + x;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double w = __shfl_xor(t, o);
      t = mn ? fmin(t, w) : t + w;
    }
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = mn ? __builtin_inf() : 0.0;
      for (int w = 0; w < kThreads / 64; ++w) r = mn ? fmin(r, lds[w]) : r + lds[w];
      out[q] = r;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_predict(const sph_soa& soa, const Prec& p, const CellsDev& c, const void* aos,
                          const AosLayout& L, double dth, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  PredIn in;
  for (int a = 0; a < 3; ++a) {
    in.v[a] = static_cast<const float*>(soa.f[SPH_S_V_X + a]);
    in.vq[a] = soa.f[SPH_S_VQ_X + a];
  }
  in.u = static_cast<const float*>(soa.f[SPH_S_UK]);
  in.uq = soa.f[SPH_S_U];
  in.vel_dt = p.vel;
  in.mhu_dt = p.mhu;
  in.store_u = p.store_u;
  in.perm = c.perm;
  in.aos = static_cast<const char*>(aos);
  in.L = L;
  k_predict<<<(c.n + kThreads - 1) / kThreads, kThreads, 0, s>>>(in, c.n, (float)dth);
  return hipGetLastError();
}

hipError_t launch_step_totals(const sph_soa& soa, const Prec& p, int n, double gamma_k,
                              double c_cfl, double* out, void* ws, hipStream_t s) {
  TotIn t;
  t.m = soa.f[SPH_S_M];
  t.h = soa.f[SPH_S_H];
  t.mhu_dt = p.mhu;
  t.lm = p.load_m;
  t.lh = p.load_h;
  for (int a = 0; a < 3; ++a) t.v[a] = static_cast<const float*>(soa.f[SPH_S_V_X + a]);
  t.u = static_cast<const float*>(soa.f[SPH_S_UK]);
  t.vsig = static_cast<const float*>(soa.f[SPH_S_VSIG]);
  t.gk = gamma_k;
  t.cfl = c_cfl;
  double* part = static_cast<double*>(ws);
  k_totals_partial<<<kReduceBlocks, kThreads, 0, s>>>(t, n, part);
  k_totals_final<<<1, kThreads, 0, s>>>(part, kReduceBlocks, out);
  return hipGetLastError();
}

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
  k_kick_drift<<<(c.n + kThreads - 1) / kThreads, kThreads, 0, s>>>(k, c.n, c.n_c, c.sub_bits,
                                                                     (float)dtk, dtd, moved);
  return hipGetLastError();
}

hipError_t launch_kick_drift_aos(void* aos, const AosLayout& L, int n, int n_c, int sub_bits,
                                 double dtk, double dtd, int32_t* moved, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_kick_drift_aos<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(
      static_cast<char*>(aos), L, n, n_c, sub_bits, (float)dtk, dtd, moved);
  return hipGetLastError();
}

size_t reduce_workspace_bytes(int n) {
  (void)n;
  return sizeof(double) * kReduceBlocks * kReduceVals;
}

// --- streaming probes of the HBM rate (the ceiling the streaming kernels are
// measured against): 16-byte non-temporal accesses, one per thread ----------
typedef float f4v __attribute__((ext_vector_type(4)));

namespace {

__global__ __launch_bounds__(kThreads) void k_probe_copy(const f4v* __restrict__ a,
                                                          f4v* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ __launch_bounds__(kThreads) void k_probe_write(f4v* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) {
    const f4v v = {1.0f, 2.0f, 3.0f, (float)i};
    __builtin_nontemporal_store(v, b + i);
  }
}

// grid-stride read, four loads in flight per thread; one word is written only
// when the sum takes a value no input here produces, so the loads stay live
__global__ __launch_bounds__(kThreads) void k_probe_read(const f4v* __restrict__ a,
                                                          float* __restrict__ sink, size_t n) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  float acc = 0.0f;
  for (; i + 3 * stride < n; i += 4 * stride) {
    f4v v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(a + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
  }
  for (; i < n; i += stride) acc += a[i].x;
  if (acc == -1.5e38f) sink[0] = acc;
}

}  // namespace

hipError_t launch_hbm_probe(int mode, const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / sizeof(f4v);
  if (n == 0) return hipSuccess;
  if (mode == SPH_PROBE_COPY) {
    k_probe_copy<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        static_cast<const f4v*>(src), static_cast<f4v*>(dst), n);
  } else if (mode == SPH_PROBE_WRITE) {
    k_probe_write<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        static_cast<f4v*>(dst), n);
  } else {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    k_probe_read<<<cus * 256, kThreads, 0, s>>>(static_cast<const f4v*>(src),
                                                static_cast<float*>(dst), n);
  }
  return hipGetLastError();
}

// Scratch of the allocation-free reduction (sph_reduce_static): the
// kReduceBlocks x kReduceVals partial sums, one copy on each device the
// library runs on. Host code never passes the array's name to a kernel: it
// resolves each device's address once, with that device current, and
// passes that address.
static __device__ __align__(256) double scratch[kReduceBlocks * kReduceVals];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t reduce_scratch_bytes() { return sizeof(scratch); }

hipError_t reduce_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
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

hipError_t launch_reduce_aos(const void* aos, const AosLayout& L, const CellsDev& c, double* out,
                             void* ws, hipStream_t s) {
  const RedAos r{static_cast<const char*>(aos), L, c.perm, c.n};
  double* part = static_cast<double*>(ws);
  k_reduce_partial<<<kReduceBlocks, kThreads, 0, s>>>(r, c.n, part);
  k_reduce_final<<<1, kThreads, 0, s>>>(part, kReduceBlocks, out);
  return hipGetLastError();
}

}  // namespace sph
