// k_dmc.hip -- diffusion Monte Carlo population control on the device (section "Diffusion
// Monte Carlo"): weights w G_B, the mixed estimator, branching M = INT(w + xi), the copies
// into free slots of a fixed-capacity population, and the trial-energy feedback.
//
// The population lives in the handle's W walker slots; a slot is alive while its weight is
// positive.  Every slot makes the step's move (dead slots move too: their results are never
// read and a slot only comes back to life as a copy, which overwrites its whole state), so
// no launch depends on the population size and a step needs nothing from the host.
#include "qmc_kernels.hpp"

namespace qmc {

constexpr int kBranchBlock = 1024;

namespace {

// Exclusive prefix sum of v over the block (kBranchBlock threads); returns the block total.
__device__ int block_exclusive_scan(int v, int* lds, int tid, int& excl) {
  lds[tid] = v;
  __syncthreads();
  for (int o = 1; o < kBranchBlock; o <<= 1) {
    const int t = tid >= o ? lds[tid - o] : 0;
    __syncthreads();
    lds[tid] += t;
    __syncthreads();
  }
  const int incl = lds[tid], total = lds[kBranchBlock - 1];
  __syncthreads();
  excl = incl - v;
  return total;
}

}  // namespace

// One workgroup.  Step k, tau = sigma^2:
//   alive slots: w <- w exp(-tau (E + E_new - 2 E_T) / 2), E <- E_new (eqs. pmc:g_growth,
//   pmc:walker_weight); E_mix = sum w E / sum w (eq. pmc:weighted_average);
//   M = floor(w + xi) capped at W (copies beyond the capacity could never be placed), xi the
//   BRANCH draw of (slot, k); dead slots M = 0;
//   free slots (M = 0) in ascending order take the extra copies (M - 1 of every slot, lower
//   slots first); a slot is alive afterwards with weight 1 if M >= 1 or it received a copy;
//   every extra copy not placed (over the free slots or over the cap) counts as dropped;
//   E_T <- E_mix - feedback ln(population / target).
// Sums are taken per thread over a strided range, then in a fixed tree: bitwise repeatable.
__global__ __launch_bounds__(kBranchBlock) void k_dmc_branch(SysParams P, DmcState D) {
  __shared__ int sscan[kBranchBlock];
  __shared__ double sred[3][kBranchBlock / 64];
  __shared__ int ired[2][kBranchBlock / 64];
  __shared__ int stot[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_of(tid);
  const int W = P.W;
  const double tau = P.sigma * P.sigma, et = D.ctl[0];
  const uint32_t step = (uint32_t)D.ictl[0];
  // (1) weights, energies, multiplicities, partial sums
  double sw = 0.0, swe = 0.0, sx = 0.0;   // sx: the extra copies asked for, before the cap
  int ncr = 0;
  for (int j = tid; j < W; j += kBranchBlock) {
    int m = 0;
    double wbj = 0.0, ebj = __builtin_nan("");
    if (D.w[j] > 0.0) {
      const double* e = D.e4 + 4 * (size_t)j;
      const double en = e[0] + e[1] + e[2] + e[3];
      const double wj = D.w[j] * exp(-tau * (D.E[j] + en - 2.0 * et) / 2.0);
      D.w[j] = wj;
      D.E[j] = en;
      sw += wj;
      swe += wj * en;
      ncr += D.crossed[j];
      double xi, unused;
      uniform_pair(P, kBranch, 0, (uint32_t)j, step, 0u, xi, unused);
      const double mr = floor(wj + xi);
      m = mr < (double)W ? (int)mr : W;
      if (mr >= 1.0) sx += mr - 1.0;
      wbj = wj;
      ebj = en;
    }
    D.mult[j] = m;
    D.wb[2 * (size_t)j] = wbj;
    D.wb[2 * (size_t)j + 1] = ebj;
  }
  sw = wave_sum_dpp(sw);
  swe = wave_sum_dpp(swe);
  sx = wave_sum_dpp(sx);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) ncr += __shfl_xor(ncr, o, 64);
  if (lane == 0) { sred[0][wave] = sw; sred[1][wave] = swe; sred[2][wave] = sx; ired[0][wave] = ncr; }
  __syncthreads();
  // (2) exclusive scans of the extra copies and of the free slots, chunk by chunk.  The copy
  // sums saturate at W: no free-slot rank reaches W, so the placement is unchanged, and a
  // chunk's sum (at most kBranchBlock (W - 1)) stays within an int.
  int carry_x = 0, carry_f = 0;
  for (int c0 = 0; c0 < W; c0 += kBranchBlock) {
    const int j = c0 + tid;
    const int m = j < W ? D.mult[j] : 1;
    const int extra = m > 1 ? m - 1 : 0, fr = (j < W && m == 0) ? 1 : 0;
    int ex, ef;
    const int tx = block_exclusive_scan(extra, sscan, tid, ex);
    const int tf = block_exclusive_scan(fr, sscan, tid, ef);
    if (j < W) { D.xscan[j] = min(carry_x + ex, W); D.fscan[j] = carry_f + ef; }
    carry_x = min(carry_x + tx, W);
    carry_f += tf;
  }
  if (tid == 0) { stot[0] = carry_x; stot[1] = carry_f; }
  __syncthreads();
  const int total_extra = stot[0], total_free = stot[1];
  // (3) plans: the r-th free slot takes extra copy r, whose source is the largest j with
  // xscan[j] <= r (that slot's extra copies cover r)
  for (int f = tid; f < W; f += kBranchBlock) {
    int src = -1;
    if (D.mult[f] == 0) {
      const int r = D.fscan[f];
      if (r < total_extra) {
        int lo = 0, hi = W - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (D.xscan[mid] <= r) lo = mid; else hi = mid - 1;
        }
        src = lo;
      }
    }
    D.plan[f] = src;
  }
  __syncthreads();
  // (4) new weights; copies take their source's energy (sources are never free slots)
  int pop = 0;
  for (int j = tid; j < W; j += kBranchBlock) {
    const int src = D.plan[j];
    const bool alive = D.mult[j] >= 1 || src >= 0;
    if (src >= 0) D.E[j] = D.E[src];
    D.w[j] = alive ? 1.0 : 0.0;
    pop += alive ? 1 : 0;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) pop += __shfl_xor(pop, o, 64);
  if (lane == 0) ired[1][wave] = pop;
  __syncthreads();
  if (tid == 0) {
    double tw = 0.0, twe = 0.0, tx = 0.0;
    int tcr = 0, tpop = 0;
    for (int q = 0; q < kBranchBlock / 64; ++q) {
      tw += sred[0][q]; twe += sred[1][q]; tx += sred[2][q]; tcr += ired[0][q]; tpop += ired[1][q];
    }
    const double emix = twe / tw;
    D.stats[0] = emix;
    D.stats[1] = tw;
    D.stats[2] = (double)tpop;
    D.stats[3] = et;
    D.stats[4] = tx - (double)(total_extra < total_free ? total_extra : total_free);
    D.stats[5] = (double)tcr;
    if (tpop == 0) D.ictl[1] = 1;   // extinct: E_T is kept
    else D.ctl[0] = emix - D.ctl[1] * log((double)tpop / (double)D.ictl[2]);
    D.ictl[0] = (int)step + 1;
  }
}

// The state of slot plan[f] copied into every slot f that received a copy: positions, row
// flags, the current rows (value, gradient, Laplacian; FP64 values, and with drift moves FP64
// gradients, in mixed precision),
// inverses, log|D| and signs.  One workgroup per slot.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmc_copy(SysParams P, Walkers<T> Wk, DmcState D) {
  const int f = blockIdx.x, tid = threadIdx.x;
  const int src = D.plan[f];
  if (src < 0) return;
  const int N = P.N;
  const size_t s0 = (size_t)src * N, f0 = (size_t)f * N;
  for (int q = tid; q < 3 * N; q += kBlock) Wk.pos[f0 * 3 + q] = Wk.pos[s0 * 3 + q];
  // rows: one wave per electron, 16-byte vectors (a row of 5 S values and an FP64 value row
  // are multiples of 16 bytes: S is padded to 16 bytes and the buffers are 256-byte aligned)
  const int lane = tid & 63, wave = wave_of(tid);
  const int rv = kComp * P.S * (int)sizeof(T) / 16, r64 = P.S * 8 / 16;
  for (int i = wave; i < N; i += kWaves) {
    const size_t b = Wk.cur[s0 + i];
    const uint4* src_row = reinterpret_cast<const uint4*>(Wk.vgl + ((b * P.W * N) + s0 + i) * kComp * P.S);
    uint4* dst_row = reinterpret_cast<uint4*>(Wk.vgl + ((b * P.W * N) + f0 + i) * kComp * P.S);
    for (int c = lane; c < rv; c += 64) dst_row[c] = src_row[c];
    if (Wk.val64) {
      const uint4* s64 = reinterpret_cast<const uint4*>(Wk.val64 + ((b * P.W * N) + s0 + i) * P.S);
      uint4* d64 = reinterpret_cast<uint4*>(Wk.val64 + ((b * P.W * N) + f0 + i) * P.S);
      for (int c = lane; c < r64; c += 64) d64[c] = s64[c];
    }
    if (Wk.grad64) {
      const uint4* s64 = reinterpret_cast<const uint4*>(Wk.grad64 + ((b * P.W * N) + s0 + i) * 3 * P.S);
      uint4* d64 = reinterpret_cast<uint4*>(Wk.grad64 + ((b * P.W * N) + f0 + i) * 3 * P.S);
      for (int c = lane; c < 3 * r64; c += 64) d64[c] = s64[c];
    }
  }
  for (size_t q = tid; q < (size_t)P.bstride; q += kBlock)
    Wk.binv[(size_t)f * P.bstride + q] = Wk.binv[(size_t)src * P.bstride + q];
  if (Wk.binv64)
    for (size_t q = tid; q < (size_t)P.bstride; q += kBlock)
      Wk.binv64[(size_t)f * P.bstride + q] = Wk.binv64[(size_t)src * P.bstride + q];
  if (D.vel)
    for (int q = tid; q < 3 * N; q += kBlock) D.vel[f0 * 3 + q] = D.vel[s0 * 3 + q];
  __syncthreads();   // every thread has read the source's row flags
  for (int i = tid; i < N; i += kBlock) Wk.cur[f0 + i] = Wk.cur[s0 + i];
  if (tid < 2) {
    Wk.logdet[2 * f + tid] = Wk.logdet[2 * src + tid];
    Wk.sign[2 * f + tid] = Wk.sign[2 * src + tid];
  }
}

hipError_t launch_dmc_branch(const SysParams& P, const DmcState& D, hipStream_t st) {
  hipLaunchKernelGGL(k_dmc_branch, dim3(1), dim3(kBranchBlock), 0, st, P, D);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dmc_copy(const SysParams& P, const Walkers<T>& Wk, const DmcState& D, hipStream_t st) {
  if (P.W <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dmc_copy<T>, dim3(P.W), dim3(kBlock), 0, st, P, Wk, D);
  return hipGetLastError();
}

template hipError_t launch_dmc_copy<float>(const SysParams&, const Walkers<float>&, const DmcState&, hipStream_t);
template hipError_t launch_dmc_copy<double>(const SysParams&, const Walkers<double>&, const DmcState&, hipStream_t);

}  // namespace qmc
