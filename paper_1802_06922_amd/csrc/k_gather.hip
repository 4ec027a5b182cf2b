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

// One table row's contribution to the five sums of an orbital, in a fixed order of fused
// multiply-adds (spelled out, so that every evaluation path rounds the same way): the z
// stencil sums s0, s1, s2 of the row's four coefficients, then the row's x-y weights.
struct RowWeights { double wab, gxab, gyab, lab; };
__device__ __forceinline__ RowWeights row_weights(double xw, double xd, double xdd, double yw, double ydw,
                                                  double yd2w) {
  return RowWeights{xw * yw, xd * yw, xw * ydw, fma(xdd, yw, xw * yd2w)};
}
__device__ __forceinline__ void row_accumulate(const Axis& az, const RowWeights& rw, double c0, double c1, double c2,
                                               double c3, double* acc, int stride) {
  const double s0 = fma(az.w[3], c3, fma(az.w[2], c2, fma(az.w[1], c1, az.w[0] * c0)));
  const double s1 = fma(az.dw[3], c3, fma(az.dw[2], c2, fma(az.dw[1], c1, az.dw[0] * c0)));
  const double s2 = fma(az.d2w[3], c3, fma(az.d2w[2], c2, fma(az.d2w[1], c1, az.d2w[0] * c0)));
  acc[0] = fma(rw.wab, s0, acc[0]);
  acc[stride] = fma(rw.gxab, s0, acc[stride]);
  acc[2 * stride] = fma(rw.gyab, s0, acc[2 * stride]);
  acc[3 * stride] = fma(rw.wab, s1, acc[3 * stride]);
  acc[4 * stride] = fma(rw.lab, s0, fma(rw.wab, s2, acc[4 * stride]));
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
  // The x-slab loop stays rolled; its weights rotate through slot 0 so every register index is
  // static.  (The compiler interleaves each row's uses with its loads here; the ordered gather
  // below keeps a whole slab's loads in flight instead.)
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
      const RowWeights rw = row_weights(xw[0], xd[0], xdd[0], ay.w[b], ay.dw[b], ay.d2w[b]);
#pragma unroll
      for (int e = 0; e < V; ++e) row_accumulate(az, rw, c0[e], c1[e], c2[e], c3[e], &acc[0][e], V);
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      xi[m] = xi[m + 1]; xw[m] = xw[m + 1]; xd[m] = xd[m + 1]; xdd[m] = xdd[m + 1];
    }
  }
}

// Buffer loads of the table: a descriptor in scalar registers and 32-bit byte offsets per lane
// (one vector register per load address instead of two).  Word 3 is the gfx9-family raw-buffer
// format; reads past the table's bytes return zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const void* table, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(table), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ void load_vec_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, double out[VecOf<T>::V]) {
  using VT = typename VecOf<T>::type;
  const auto raw = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
  const VT v = __builtin_bit_cast(VT, raw);
  const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
  for (int k = 0; k < VecOf<T>::V; ++k) out[k] = (double)e[k];
}

// The same sums with the item's x and y weights read from LDS (one copy per item instead of one
// per lane) and the table read by buffer loads: the registers this frees keep more loads in
// flight.  The rounding steps are those of spline_vgl_vec (row_weights, row_accumulate), so
// the results are bitwise the same.  The table must hold fewer than 2^32 bytes.
template <typename T>
__device__ __forceinline__ void spline_vgl_vec_xy(__amdgpu_buffer_rsrc_t rs, const SysParams& P, const Axis& ax,
                                                  const Axis& ay, const Axis& az, int q,
                                                  double acc[kComp][VecOf<T>::V]) {
  constexpr int V = VecOf<T>::V;
#pragma unroll
  for (int c = 0; c < kComp; ++c)
#pragma unroll
    for (int e = 0; e < V; ++e) acc[c][e] = 0.0;
  const uint32_t zs = (uint32_t)P.S * sizeof(T);
  const uint32_t qo = (uint32_t)q * V * sizeof(T);
  uint32_t zo[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) zo[m] = (uint32_t)az.idx[m] * zs + qo;
#pragma unroll 1
  for (int a = 0; a < 4; ++a) {
    const uint32_t xbase = (uint32_t)ax.idx[a] * P.gy;
    const double xw = ax.w[a], xd = ax.dw[a], xdd = ax.d2w[a];
    double c0[4][V], c1[4][V], c2[4][V], c3[4][V];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t row = (xbase + (uint32_t)ay.idx[b]) * (uint32_t)P.gz * zs;
      load_vec_buf<T>(rs, row + zo[0], c0[b]);
      load_vec_buf<T>(rs, row + zo[1], c1[b]);
      load_vec_buf<T>(rs, row + zo[2], c2[b]);
      load_vec_buf<T>(rs, row + zo[3], c3[b]);
    }
    // the slab's 16 loads are issued before any of them is used (else the scheduler puts each
    // use right after its load and the wave waits out every round trip in turn)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const RowWeights rw = row_weights(xw, xd, xdd, ay.w[b], ay.dw[b], ay.d2w[b]);
#pragma unroll
      for (int e = 0; e < V; ++e) row_accumulate(az, rw, c0[b][e], c1[b][e], c2[b][e], c3[b][e], &acc[0][e], V);
    }
  }
}

// Proposal of item (walker w, electron i) in sweep `sweep` (section "Trial Moves"): r' and its
// acceptance uniform from the counter-based streams of (w, sweep, i).
template <typename T>
__device__ __forceinline__ void propose_item(const SysParams& P, const Walkers<T>& Wk, long item, uint32_t sweep,
                                             double r[3], double& u0) {
#pragma clang fp contract(off)   // the same bits in every kernel that draws proposals
  const int w = (int)(item / P.N), i = (int)(item % P.N);
  const double* p0 = Wk.pos + item * 3;
  double a0, a1, b0, b1, u1;
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
}

// The rows of vector q of item (values, gradients, Laplacians; FP64 copies where kept).
template <typename T>
__device__ __forceinline__ void store_item_vec(const SysParams& P, const Walkers<T>& Wk, long item, int buf, int q,
                                               const double acc[kComp][VecOf<T>::V]) {
  constexpr int V = VecOf<T>::V;
  T* out = Wk.vgl + ((size_t)buf * P.W * P.N + (size_t)item) * kComp * P.S;
#pragma unroll
  for (int c = 0; c < kComp; ++c) store_vec<T>(out + (size_t)c * P.S + (size_t)q * V, acc[c]);
  if (Wk.val64) {   // mixed precision keeps the FP64 values for re-decisions and rebuilds
    double* out64 = Wk.val64 + ((size_t)buf * P.W * P.N + (size_t)item) * P.S;
#pragma unroll
    for (int e = 0; e < V; ++e) out64[(size_t)q * V + e] = acc[0][e];
  }
  if (Wk.grad64) {  // and, with drift moves, the FP64 gradients the velocities are built from
    double* g64 = Wk.grad64 + ((size_t)buf * P.W * P.N + (size_t)item) * 3 * P.S;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < V; ++e) g64[(size_t)c * P.S + (size_t)q * V + e] = acc[1 + c][e];
  }
}

// Value, gradient and Laplacian rows of item at r, into row buffer buf; tpi lanes per item.
template <typename T>
__device__ __forceinline__ void evaluate_item(const SysParams& P, const Walkers<T>& Wk, const T* __restrict__ table,
                                              long item, const double r[3], int buf, int lane, int tpi) {
  constexpr int V = VecOf<T>::V;
  Axis ax, ay, az;
  axis_weights(r[0], P.L, P.gx, ax);
  axis_weights(r[1], P.L, P.gy, ay);
  axis_weights(r[2], P.L, P.gz, az);
  const int nvec = P.S / V;
  for (int q = lane; q < nvec; q += tpi) {
    double acc[kComp][V];
    spline_vgl_vec<T>(table, P, ax, ay, az, q, acc);
    store_item_vec<T>(P, Wk, item, buf, q, acc);
  }
}

// One item = one (walker, electron); tpi = 1 << tpi_log2 lanes per item.
template <typename T>
__device__ __forceinline__ void gather_item(const SysParams& P, const Walkers<T>& Wk,
                                            const T* __restrict__ table, int mode, long item, int lane,
                                            int tpi, const uint32_t* sel = nullptr, uint32_t sel_value = 0) {
  if (item >= (long)P.W * P.N) return;
  const int w = (int)(item / P.N);
  if (sel && sel[w] != sel_value) return;   // (lanes work independently: no wave operations below)
  double r[3];
  int buf;
  if (mode == 0) {
    double u0;
    propose_item<T>(P, Wk, item, *Wk.sweep_ctr, r, u0);
    if (lane == 0) {
      double* pr = Wk.prop + item * 4;
      pr[0] = r[0]; pr[1] = r[1]; pr[2] = r[2]; pr[3] = u0;
    }
    buf = 1 - (int)Wk.cur[item];
  } else {
    const double* p0 = Wk.pos + item * 3;
    r[0] = p0[0]; r[1] = p0[1]; r[2] = p0[2];
    buf = 0;
    if (lane == 0) Wk.cur[item] = 0;
  }
  evaluate_item<T>(P, Wk, table, item, r, buf, lane, tpi);
}

// ---------------------------------------------------------------------------
// The sweep's proposals in table order.  Every proposal reads a 4 x 4 x 4 block of table
// points, and a sweep's proposals touch each point about 64 N W / (gx gy gz) times; in
// (walker, electron) order those reads are scattered over the whole table and miss the
// caches.  The proposals are therefore drawn first (one thread each), bucketed by the table
// tile that holds them (tiles in Morton order, so consecutive buckets are neighbours),
// counting-sorted, and evaluated in bucket order, with the workgroups of each XCD (block
// index mod 8) taking one contiguous slice of the order: the proposals in flight on an XCD
// then share most of their table blocks in that XCD's L2.  Each item's arithmetic is the
// same as in (walker, electron) order, so the rows are bitwise the same.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int gather_bucket(const SysParams& P, const GatherOrder& G, const double r[3]) {
  const int g[3] = {P.gx, P.gy, P.gz};
  int key = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int c = (int)(r[a] / P.L * g[a]);
    c = c < 0 ? 0 : (c >= g[a] ? g[a] - 1 : c);
    const int t = c / G.tile[a];   // < 16
#pragma unroll
    for (int b = 0; b < 4; ++b) key |= ((t >> b) & 1) << (3 * b + a);
  }
  return key;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_propose(SysParams P, Walkers<T> Wk, GatherOrder G) {
  const long item = (long)blockIdx.x * kBlock + threadIdx.x;
  if (item >= (long)P.W * P.N) return;
  double r[3], u0;
  propose_item<T>(P, Wk, item, *Wk.sweep_ctr, r, u0);
  double* pr = Wk.prop + item * 4;
  pr[0] = r[0]; pr[1] = r[1]; pr[2] = r[2]; pr[3] = u0;
  const int key = gather_bucket(P, G, r);
  G.key[item] = key;
  atomicAdd(G.hist + key, 1);
}

// Exclusive scan of the bucket counts into the bucket starts (one workgroup); the counts are
// cleared for the next sweep.
__global__ __launch_bounds__(kBlock) void k_bucket_scan(GatherOrder G) {
  constexpr int kPer = kGatherBuckets / kBlock;
  static_assert(kPer * kBlock == kGatherBuckets, "buckets split evenly over the threads");
  __shared__ int part[kBlock];
  const int t = threadIdx.x;
  int c[kPer], sum = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    c[e] = G.hist[t * kPer + e];
    sum += c[e];
  }
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {   // inclusive scan of the per-thread sums
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    G.offs[t * kPer + e] = run;
    run += c[e];
    G.hist[t * kPer + e] = 0;
  }
}

// Each item takes the next free place of its bucket (the order within a bucket is free: the
// items are independent).
__global__ __launch_bounds__(kBlock) void k_bucket_scatter(long n_items, GatherOrder G) {
  const long item = (long)blockIdx.x * kBlock + threadIdx.x;
  if (item >= n_items) return;
  const int slot = atomicAdd(G.offs + G.key[item], 1);
  if (slot < n_items) G.order[slot] = (int)item;
}

// Evaluation in bucket order: chunk c (kBlock >> tpi_log2 consecutive places of the order) runs
// on block b with b mod 8 = c / per_xcd, the XCD that block b is dispatched to.  The x and y
// weights of each item go to LDS (dynamic: 2 Axis per item).
template <typename T>
__global__ __launch_bounds__(kBlock, 2) void k_gather_ordered(SysParams P, Walkers<T> Wk, const T* __restrict__ table,
                                                           int tpi_log2, GatherOrder G, int n_chunks, int per_xcd) {
  constexpr int V = VecOf<T>::V;
  extern __shared__ Axis sxy[];   // [items per block][2]
  const int chunk = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (chunk >= n_chunks) return;   // the whole block
  const int tpi = 1 << tpi_log2, lane = threadIdx.x & (tpi - 1), slot = threadIdx.x >> tpi_log2;
  const long place = (long)chunk * (kBlock >> tpi_log2) + slot;
  long item = -1;
  if (place < (long)P.W * P.N) {
    item = G.order[place];
    if (item < 0 || item >= (long)P.W * P.N) item = -1;
  }
  Axis az;
  if (item >= 0) {
    const double* pr = Wk.prop + item * 4;
    if (lane == 0) axis_weights(pr[0], P.L, P.gx, sxy[2 * slot]);
    if (lane == (tpi > 1 ? 1 : 0)) axis_weights(pr[1], P.L, P.gy, sxy[2 * slot + 1]);
    axis_weights(pr[2], P.L, P.gz, az);
  }
  __syncthreads();
  if (item < 0) return;
  const int buf = 1 - (int)Wk.cur[item];
  const int nvec = P.S / V;
  const __amdgpu_buffer_rsrc_t rs = table_rsrc(table, (uint32_t)((size_t)P.gx * P.gy * P.gz * P.S * sizeof(T)));
  for (int q = lane; q < nvec; q += tpi) {
    double acc[kComp][V];
    spline_vgl_vec_xy<T>(rs, P, sxy[2 * slot], sxy[2 * slot + 1], az, q, acc);
    store_item_vec<T>(P, Wk, item, buf, q, acc);
  }
}

// The sweep's proposals (mode 0), in (walker, electron) order.
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
                         int lanes_log2, const uint32_t* sel, uint32_t sel_value, const GatherOrder* go) {
  const int nvec = P.S / VecOf<T>::V;
  const int tl = lanes_log2 >= 0 && lanes_log2 <= 6 ? lanes_log2 : gather_tpi_log2(nvec);
  const long items = (long)P.W * P.N;
  const long per_block = kBlock >> tl;
  const unsigned blocks = (unsigned)((items + per_block - 1) / per_block);
  // (the ordered kernel addresses the table in 32-bit byte offsets)
  if (mode == 0 && go && (double)P.gx * P.gy * P.gz * P.S * sizeof(T) < 4294967296.0) {
    const unsigned iblocks = (unsigned)((items + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_propose<T>, dim3(iblocks), dim3(kBlock), 0, st, P, Wk, *go);
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(kBlock), 0, st, *go);
    hipLaunchKernelGGL(k_bucket_scatter, dim3(iblocks), dim3(kBlock), 0, st, items, *go);
    const int per_xcd = (int)((blocks + 7) / 8);
    hipLaunchKernelGGL(k_gather_ordered<T>, dim3(8 * per_xcd), dim3(kBlock), 2 * per_block * sizeof(Axis), st, P,
                       Wk, table, tl, *go, (int)blocks, per_xcd);
  } else if (mode == 0)
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
                                          hipStream_t, int, const uint32_t*, uint32_t, const GatherOrder*);
template hipError_t launch_gather<float>(const SysParams&, const Walkers<float>&, const float*, int,
                                         hipStream_t, int, const uint32_t*, uint32_t, const GatherOrder*);
template hipError_t launch_gather_batched<double>(const SysDev<double>*, const int2*, int, hipStream_t);
template hipError_t launch_gather_batched<float>(const SysDev<float>*, const int2*, int, hipStream_t);
template hipError_t launch_eval_points<double>(const SysParams&, const double*, const double*, int,
                                               double*, hipStream_t);
template hipError_t launch_eval_points<float>(const SysParams&, const float*, const double*, int,
                                              double*, hipStream_t);

}  // namespace qmc
