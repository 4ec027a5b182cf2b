// k_gather.hip -- proposal generation and periodic tricubic B-spline orbital
// evaluation (value, gradient, Laplacian) for every (walker, electron).
//
// Section "B-spline basis sets": each orbital value needs 64 coefficients
// (the 4x4x4 stencil of the cell holding the point), independent of the
// basis size.  The table is stored orbital-contiguous, C[ix][iy][iz][S], so
// one stencil point is one contiguous run of S coefficients: the lanes of an
// item read consecutive 16-byte vectors of orbitals (coalesced), and the 4
// z-neighbours of an (ix, iy) row are S apart.
//
// Every proposal of a sweep depends only on the proposing electron's own
// position (section "Trial Moves": r' = r_i + sigma xi, no drift), and
// electron i's position changes only at its own move, so the orbital rows of
// all N proposals of all walkers are evaluated here in one fully parallel
// launch before the sequential move chain runs.
#include "qmc_kernels.hpp"

namespace qmc {

template <typename T> struct VecOf;
template <> struct VecOf<double> { using type = double2; static constexpr int V = 2; };
template <> struct VecOf<float> { using type = float4; static constexpr int V = 4; };

template <typename T>
__device__ __forceinline__ void load_vec(const T* p, double out[VecOf<T>::V]) {
  using VT = typename VecOf<T>::type;
  const VT v = *reinterpret_cast<const VT*>(p);
  const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
  for (int k = 0; k < VecOf<T>::V; ++k) out[k] = (double)e[k];
}

template <typename T>
__device__ __forceinline__ void store_vec(T* p, const double in[VecOf<T>::V]) {
  using VT = typename VecOf<T>::type;
  VT v;
  T* e = reinterpret_cast<T*>(&v);
#pragma unroll
  for (int k = 0; k < VecOf<T>::V; ++k) e[k] = (T)in[k];
  *reinterpret_cast<VT*>(p) = v;
}

// Value, gradient and Laplacian of the V orbitals of vector q.
template <typename T>
__device__ __forceinline__ void spline_vgl_vec(const T* __restrict__ table, const SysParams& P,
                                               const Axis& ax, const Axis& ay, const Axis& az, int q,
                                               double acc[kComp][VecOf<T>::V]) {
  constexpr int V = VecOf<T>::V;
#pragma unroll
  for (int c = 0; c < kComp; ++c)
#pragma unroll
    for (int e = 0; e < V; ++e) acc[c][e] = 0.0;
  const size_t zs = (size_t)P.S;
  // The x-slab loop stays rolled (each iteration issues the 16 loads of one
  // slab at once); its weights rotate through slot 0 so every register index
  // is static.
  int xi[4] = {ax.idx[0], ax.idx[1], ax.idx[2], ax.idx[3]};
  double xw[4] = {ax.w[0], ax.w[1], ax.w[2], ax.w[3]};
  double xd[4] = {ax.dw[0], ax.dw[1], ax.dw[2], ax.dw[3]};
  double xdd[4] = {ax.d2w[0], ax.d2w[1], ax.d2w[2], ax.d2w[3]};
#pragma unroll 1
  for (int a = 0; a < 4; ++a) {
    const size_t xbase = (size_t)xi[0] * P.gy;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const T* row = table + ((xbase + ay.idx[b]) * P.gz) * zs + (size_t)q * V;
      double c0[V], c1[V], c2[V], c3[V];
      load_vec<T>(row + az.idx[0] * zs, c0);
      load_vec<T>(row + az.idx[1] * zs, c1);
      load_vec<T>(row + az.idx[2] * zs, c2);
      load_vec<T>(row + az.idx[3] * zs, c3);
      const double wab = xw[0] * ay.w[b];
      const double gxab = xd[0] * ay.w[b];
      const double gyab = xw[0] * ay.dw[b];
      const double lab = xdd[0] * ay.w[b] + xw[0] * ay.d2w[b];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const double s0 = az.w[0] * c0[e] + az.w[1] * c1[e] + az.w[2] * c2[e] + az.w[3] * c3[e];
        const double s1 = az.dw[0] * c0[e] + az.dw[1] * c1[e] + az.dw[2] * c2[e] + az.dw[3] * c3[e];
        const double s2 = az.d2w[0] * c0[e] + az.d2w[1] * c1[e] + az.d2w[2] * c2[e] + az.d2w[3] * c3[e];
        acc[0][e] += wab * s0;
        acc[1][e] += gxab * s0;
        acc[2][e] += gyab * s0;
        acc[3][e] += wab * s1;
        acc[4][e] += lab * s0 + wab * s2;
      }
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      xi[m] = xi[m + 1]; xw[m] = xw[m + 1]; xd[m] = xd[m + 1]; xdd[m] = xdd[m + 1];
    }
  }
}

// One item = one (walker, electron); tpi = 1 << tpi_log2 lanes per item.
template <typename T>
__device__ __forceinline__ void gather_item(const SysParams& P, const Walkers<T>& Wk,
                                            const T* __restrict__ table, int mode, long item, int lane,
                                            int tpi, const uint32_t* sel = nullptr, uint32_t sel_value = 0) {
  constexpr int V = VecOf<T>::V;
  if (item >= (long)P.W * P.N) return;
  const uint32_t sweep = mode == 0 ? *Wk.sweep_ctr : 0u;
  const int w = (int)(item / P.N), i = (int)(item % P.N);
  if (sel && sel[w] != sel_value) return;   // (lanes work independently: no wave operations below)
  const double* p0 = Wk.pos + item * 3;
  double r[3];
  int buf;
  if (mode == 0) {
    double a0, a1, b0, b1, u0, u1;
    uniform_pair(P, kPropose, 0, (uint32_t)w, sweep, (uint32_t)i, a0, a1);
    uniform_pair(P, kPropose, 1, (uint32_t)w, sweep, (uint32_t)i, b0, b1);
    uniform_pair(P, kAccept, 0, (uint32_t)w, sweep, (uint32_t)i, u0, u1);
    const double ra = sqrt(-2.0 * log(1.0 - a0));
    const double rb = sqrt(-2.0 * log(1.0 - b0));
    double sa, ca;
    sincos(2.0 * kPi * a1, &sa, &ca);
    const double cb = cos(2.0 * kPi * b1);
    if (Wk.drift_v) {
      // drift-diffusion proposal: mean r + tau v with tau = sigma^2 (variance tau per coordinate)
      const double* v = Wk.drift_v + item * 3;
      const double tau = P.sigma * P.sigma;
      r[0] = wrap_cell(p0[0] + tau * v[0] + P.sigma * (ra * ca), P.L);
      r[1] = wrap_cell(p0[1] + tau * v[1] + P.sigma * (ra * sa), P.L);
      r[2] = wrap_cell(p0[2] + tau * v[2] + P.sigma * (rb * cb), P.L);
    } else {
      r[0] = wrap_cell(p0[0] + P.sigma * (ra * ca), P.L);
      r[1] = wrap_cell(p0[1] + P.sigma * (ra * sa), P.L);
      r[2] = wrap_cell(p0[2] + P.sigma * (rb * cb), P.L);
    }
    if (lane == 0) {
      double* pr = Wk.prop + item * 4;
      pr[0] = r[0]; pr[1] = r[1]; pr[2] = r[2]; pr[3] = u0;
    }
    buf = 1 - (int)Wk.cur[item];
  } else {
    r[0] = p0[0]; r[1] = p0[1]; r[2] = p0[2];
    buf = 0;
    if (lane == 0) Wk.cur[item] = 0;
  }
  Axis ax, ay, az;
  axis_weights(r[0], P.L, P.gx, ax);
  axis_weights(r[1], P.L, P.gy, ay);
  axis_weights(r[2], P.L, P.gz, az);
  T* out = Wk.vgl + ((size_t)buf * P.W * P.N + (size_t)item) * kComp * P.S;
  double* out64 = Wk.val64 ? Wk.val64 + ((size_t)buf * P.W * P.N + (size_t)item) * P.S : nullptr;
  double* g64 = Wk.grad64 ? Wk.grad64 + ((size_t)buf * P.W * P.N + (size_t)item) * 3 * P.S : nullptr;
  const int nvec = P.S / V;
  for (int q = lane; q < nvec; q += tpi) {
    double acc[kComp][V];
    spline_vgl_vec<T>(table, P, ax, ay, az, q, acc);
#pragma unroll
    for (int c = 0; c < kComp; ++c) store_vec<T>(out + (size_t)c * P.S + (size_t)q * V, acc[c]);
    if (out64) {   // mixed precision keeps the FP64 values for re-decisions and rebuilds
#pragma unroll
      for (int e = 0; e < V; ++e) out64[(size_t)q * V + e] = acc[0][e];
    }
    if (g64)       // and, with drift moves, the FP64 gradients the velocities are built from
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int e = 0; e < V; ++e) g64[(size_t)c * P.S + (size_t)q * V + e] = acc[1 + c][e];
  }
}

// The sweep's proposals (mode 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(SysParams P, Walkers<T> Wk, const T* __restrict__ table,
                                                   int tpi_log2) {
  const long item = (long)blockIdx.x * (kBlock >> tpi_log2) + (threadIdx.x >> tpi_log2);
  gather_item<T>(P, Wk, table, 0, item, threadIdx.x & ((1 << tpi_log2) - 1), 1 << tpi_log2);
}

// Rows at the current positions (mode 1: walker initialisation), optionally for the selected
// walkers only; a kernel of its own so that profiles keep it apart from the sweeps.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_current(SysParams P, Walkers<T> Wk, const T* __restrict__ table,
                                                           int tpi_log2, const uint32_t* sel, uint32_t sel_value) {
  const long item = (long)blockIdx.x * (kBlock >> tpi_log2) + (threadIdx.x >> tpi_log2);
  gather_item<T>(P, Wk, table, 1, item, threadIdx.x & ((1 << tpi_log2) - 1), 1 << tpi_log2, sel, sel_value);
}

// Several systems in one launch: block b works on items bmap[b].y .. of system bmap[b].x.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_batched(const SysDev<T>* __restrict__ sd,
                                                           const int2* __restrict__ bmap) {
  __shared__ SysDev<T> s;
  const int2 m = bmap[blockIdx.x];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(sd + m.x);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&s);
    for (int q = threadIdx.x; q < (int)(sizeof(SysDev<T>) / 4); q += kBlock) dst[q] = src[q];
  }
  __syncthreads();
  const int tl = s.tpi_log2;
  const long item = (long)m.y + (threadIdx.x >> tl);
  gather_item<T>(s.P, s.W, s.table, 0, item, threadIdx.x & ((1 << tl) - 1), 1 << tl);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_eval_points(SysParams P, const T* __restrict__ table,
                                                        const double* __restrict__ pos, int n,
                                                        double* __restrict__ out) {
  constexpr int V = VecOf<T>::V;
  const int nvec = P.S / V;
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long)n * nvec) return;
  const int p = (int)(t / nvec), q = (int)(t % nvec);
  Axis ax, ay, az;
  axis_weights(pos[3 * p + 0], P.L, P.gx, ax);
  axis_weights(pos[3 * p + 1], P.L, P.gy, ay);
  axis_weights(pos[3 * p + 2], P.L, P.gz, az);
  double acc[kComp][V];
  spline_vgl_vec<T>(table, P, ax, ay, az, q, acc);
  for (int c = 0; c < kComp; ++c)
    for (int e = 0; e < V; ++e) {
      const int j = q * V + e;
      if (j < P.n_orb) out[((size_t)p * kComp + c) * P.n_orb + j] = acc[c][e];
    }
}

// Uniform starting positions: electron i of walker w from the INIT counters (i, 0, w).
__global__ __launch_bounds__(kBlock) void k_init_positions(SysParams P, double* __restrict__ pos) {
  const long item = (long)blockIdx.x * kBlock + threadIdx.x;
  if (item >= (long)P.W * P.N) return;
  const int w = (int)(item / P.N), i = (int)(item % P.N);
  double a0, a1, b0, b1;
  uniform_pair(P, kInit, 0, (uint32_t)w, 0u, (uint32_t)i, a0, a1);
  uniform_pair(P, kInit, 1, (uint32_t)w, 0u, (uint32_t)i, b0, b1);
  pos[item * 3 + 0] = wrap_cell(P.L * a0, P.L);
  pos[item * 3 + 1] = wrap_cell(P.L * a1, P.L);
  pos[item * 3 + 2] = wrap_cell(P.L * b0, P.L);
}

// Default lanes per proposal: 16 once a stencil point has at least 16 vectors (measured
// best at 32 and 48 vectors: fuller passes than 32 or 64 lanes leave), else the smallest
// power of two that covers the row.
int gather_tpi_log2(int nvec) {
  if (nvec >= 16) return 4;
  int l = 0;
  while ((1 << l) < nvec && l < 6) ++l;
  return l;
}

template <typename T>
hipError_t launch_gather(const SysParams& P, const Walkers<T>& Wk, const T* table, int mode, hipStream_t st,
                         int lanes_log2, const uint32_t* sel, uint32_t sel_value) {
  const int nvec = P.S / VecOf<T>::V;
  const int tl = lanes_log2 >= 0 && lanes_log2 <= 6 ? lanes_log2 : gather_tpi_log2(nvec);
  const long items = (long)P.W * P.N;
  const long per_block = kBlock >> tl;
  const unsigned blocks = (unsigned)((items + per_block - 1) / per_block);
  if (mode == 0)
    hipLaunchKernelGGL(k_gather<T>, dim3(blocks), dim3(kBlock), 0, st, P, Wk, table, tl);
  else
    hipLaunchKernelGGL(k_gather_current<T>, dim3(blocks), dim3(kBlock), 0, st, P, Wk, table, tl, sel, sel_value);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_batched(const SysDev<T>* sd, const int2* bmap, int n_blocks, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_batched<T>, dim3(n_blocks), dim3(kBlock), 0, st, sd, bmap);
  return hipGetLastError();
}

int gather_items_per_block(int S, size_t tsize) {
  return kBlock >> gather_tpi_log2(S / (tsize == sizeof(double) ? 2 : 4));
}

template <typename T>
hipError_t launch_eval_points(const SysParams& P, const T* table, const double* pos, int n,
                              double* out, hipStream_t st) {
  const long threads = (long)n * (P.S / VecOf<T>::V);
  const unsigned blocks = (unsigned)((threads + kBlock - 1) / kBlock);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_points<T>, dim3(blocks), dim3(kBlock), 0, st, P, table, pos, n, out);
  return hipGetLastError();
}

hipError_t launch_init_positions(const SysParams& P, double* pos, hipStream_t st) {
  const long items = (long)P.W * P.N;
  const unsigned blocks = (unsigned)((items + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_init_positions, dim3(blocks), dim3(kBlock), 0, st, P, pos);
  return hipGetLastError();
}

template hipError_t launch_gather<double>(const SysParams&, const Walkers<double>&, const double*, int,
                                          hipStream_t, int, const uint32_t*, uint32_t);
template hipError_t launch_gather<float>(const SysParams&, const Walkers<float>&, const float*, int,
                                         hipStream_t, int, const uint32_t*, uint32_t);
template hipError_t launch_gather_batched<double>(const SysDev<double>*, const int2*, int, hipStream_t);
template hipError_t launch_gather_batched<float>(const SysDev<float>*, const int2*, int, hipStream_t);
template hipError_t launch_eval_points<double>(const SysParams&, const double*, const double*, int,
                                               double*, hipStream_t);
template hipError_t launch_eval_points<float>(const SysParams&, const float*, const double*, int,
                                              double*, hipStream_t);

}  // namespace qmc
