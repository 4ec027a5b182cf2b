// k_allelectron.hip -- all-electron moves: every electron of a walker is proposed at once
// (section "Trial Moves", the move that displaces all coordinates together) and the walker
// accepts with min(1, |Psi(R')/Psi(R)|^2).
//
// The proposals and their value rows come from the sweep gather (the rows land in the
// buffers that do not hold the current rows).  The determinants at R' are fresh FP64
// Gauss-Jordan eliminations of those rows (the rebuild kernels, pointed at the other row
// buffer and at side outputs), so |D(R')/D(R)| = exp(log|D'| - log|D|) per spin.  This file
// adds the full Jastrow change and the per-walker decision that installs the new state.
#include "qmc_kernels.hpp"

namespace qmc {

namespace {

__device__ __forceinline__ double ae_u(const Jastrow& J, int kind, double r) {
  return kind == 0 ? radial_value(J.same, r) : (kind == 1 ? radial_value(J.opp, r) : radial_value(J.ei, r));
}

__device__ __forceinline__ double ae_dist(const double* a, const double* b, double L, double invL) {
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  const double x = dx - L * rint(dx * invL), y = dy - L * rint(dy * invL), z = dz - L * rint(dz * invL);
  return sqrt(x * x + y * y + z * z);
}

}  // namespace

// dJ[w] = J(R') - J(R), J = sum_{i<j} u2(r_ij) + sum_{i,I} u1(r_iI) (+ the three-body terms)
// (section "Jastrow factors", minimum image), as the sum of the per-pair changes.  Workgroup
// (w, p) of jastrow_parts(N) per walker takes the p-th contiguous share of each item list and
// writes dj[w * parts + p]; the decision adds the parts in order.
// The N(N-1)/2 pairs are enumerated as circulant diagonals, pair (i, i + d mod N) for
// d = 1 .. (N-1)/2 and, for even N, (i, i + N/2) with i < N/2, so the work is balanced
// over the threads without a triangular index decode.  Also clears status_prop[w], which the
// rebuild of the proposed matrices then sets on a singular matrix.
__global__ __launch_bounds__(kBlock) void k_ae_jastrow(SysParams P, const double* __restrict__ pos,
                                                       const double* __restrict__ prop, double* dj,
                                                       int* status_prop) {
  __shared__ Jastrow sj;
  __shared__ double red[kWaves];
  const int parts = gridDim.x / P.W;
  const int w = blockIdx.x / parts, p = blockIdx.x - w * parts;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_of(tid);
  const int N = P.N;
  for (int q = tid; q < (int)(sizeof(Jastrow) / sizeof(double)); q += kBlock)
    reinterpret_cast<double*>(&sj)[q] = reinterpret_cast<const double*>(&P.jas)[q];
  __syncthreads();
  const double L = P.L, invL = 1.0 / P.L;
  const double* x0 = pos + (size_t)w * N * 3;
  const double* x1 = prop + (size_t)w * N * 4;
  const int D = (N - 1) / 2;
  const int n_pairs = N * D + ((N & 1) ? 0 : N / 2);
  double acc = 0.0;
  const int q0 = (int)((long)n_pairs * p / parts), q1 = (int)((long)n_pairs * (p + 1) / parts);
  for (int q = q0 + tid; q < q1; q += kBlock) {
    int i, j;
    if (q < N * D) {
      const int d = 1 + q / N;
      i = q - (d - 1) * N;
      j = i + d;
      if (j >= N) j -= N;
    } else {
      i = q - N * D;
      j = i + N / 2;
    }
    const int kind = ((i < P.n_up) == (j < P.n_up)) ? 0 : 1;
    const double r1 = ae_dist(x1 + 4 * i, x1 + 4 * j, L, invL);
    const double r0 = ae_dist(x0 + 3 * i, x0 + 3 * j, L, invL);
    acc += ae_u(sj, kind, r1) - ae_u(sj, kind, r0);
  }
  const int ne = N * P.n_ions;
  const int e0 = (int)((long)ne * p / parts), e1 = (int)((long)ne * (p + 1) / parts);
  if (sj.ei.kind != QMC_J_NONE)
    for (int q = e0 + tid; q < e1; q += kBlock) {
      const int i = q / P.n_ions, I = q - i * P.n_ions;
      const double* ion = P.ions + 4 * I;
      acc += ae_u(sj, 2, ae_dist(x1 + 4 * i, ion, L, invL)) - ae_u(sj, 2, ae_dist(x0 + 3 * i, ion, L, invL));
    }
  if (P.j3_on) {
    // three-body terms: (ion, electron i) items, partners j > i near the same ion
    const double h = P.j3_h;
    for (int q = e0 + tid; q < e1; q += kBlock) {
      const int I = q / N, i = q - I * N;
      const double* ion = P.ions + 4 * I;
      const double a1 = ae_dist(x1 + 4 * i, ion, L, invL), a0 = ae_dist(x0 + 3 * i, ion, L, invL);
      if (a1 >= h && a0 >= h) continue;
      const bool up_i = i < P.n_up;
      for (int j = i + 1; j < N; ++j) {
        const double b1 = ae_dist(x1 + 4 * j, ion, L, invL), b0 = ae_dist(x0 + 3 * j, ion, L, invL);
        const bool same = up_i == (j < P.n_up);
        if (a1 < h && b1 < h) acc += u3_value(P, same, a1, b1, ae_dist(x1 + 4 * i, x1 + 4 * j, L, invL));
        if (a0 < h && b0 < h) acc -= u3_value(P, same, a0, b0, ae_dist(x0 + 3 * i, x0 + 3 * j, L, invL));
      }
    }
  }
  acc = wave_sum_dpp(acc);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) s += red[q];   // fixed order: bitwise repeatable
    dj[(size_t)w * parts + p] = s;
    if (p == 0) status_prop[w] = 0;
  }
}

// Drift velocities v_i = grad_i ln|Psi| = sum_l grad phi_l(r_i) B[l][k] + grad_i J of every
// electron.  prop = 0: the current configuration R (current rows, Wk.binv, Wk.pos) into vel;
// prop = 1: the proposed R' (the other row buffer, the inverses A.binv at R', the proposals)
// into vel, and then the log of the transition ratio T(R' -> R) / T(R -> R') of the
// drift-diffusion proposal (tau = sigma^2, unwrapped displacement R' - R = tau v(R) + sigma xi,
// xi redrawn from the sweep's PROPOSE counters):
//   logT = sum_i [ |sigma xi_i|^2 - |sigma xi_i + tau (v_i(R) + v_i(R'))|^2 ] / (2 tau),
// v(R) read from vcur, one partial sum per workgroup in A.logT[w * parts + p].
// Grid: (walker, part) with kVelE electrons per part; four lanes per electron split the
// orbital sum and the partner sum (every fourth term) and add them by lane shuffles.
constexpr int kVelMaxN = 1024;
constexpr int kVelE = kBlock / 4;   // electrons per workgroup

int velocity_parts(int N) { return (N + kVelE - 1) / kVelE; }

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ae_velocity(SysParams P, Walkers<T> Wk, AeProposal<T> A, int prop,
                                                        double* vel, const double* vcur) {
  __shared__ Jastrow sj;
  __shared__ double sx[kVelMaxN], sy[kVelMaxN], sz[kVelMaxN];
  __shared__ double red[kWaves];
  const int parts = gridDim.x / P.W;
  const int w = blockIdx.x / parts, p = blockIdx.x - w * parts;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_of(tid);
  const int s = tid & 3, i = p * kVelE + (tid >> 2);
  const int N = P.N;
  const bool valid = i < N;
  for (int q = tid; q < (int)(sizeof(Jastrow) / sizeof(double)); q += kBlock)
    reinterpret_cast<double*>(&sj)[q] = reinterpret_cast<const double*>(&P.jas)[q];
  const double* x = prop ? Wk.prop + (size_t)w * N * 4 : Wk.pos + (size_t)w * N * 3;
  const int xs = prop ? 4 : 3;
  for (int q = tid; q < N; q += kBlock) {
    sx[q] = x[(size_t)q * xs]; sy[q] = x[(size_t)q * xs + 1]; sz[q] = x[(size_t)q * xs + 2];
  }
  __syncthreads();
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  if (valid) {
    // determinant part: orbitals l = s, s + 4, ...
    const int sp = i < P.n_up ? 0 : 1;
    const int n = sp ? P.n_dn : P.n_up, k = i - (sp ? P.n_up : 0);
    const size_t item = (size_t)w * N + i;
    const int buf = Wk.cur[item] ^ prop;
    const size_t boff = (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0) + k;
    if (Wk.grad64) {
      // mixed precision: FP64 gradient rows and the FP64 inverse, so the proposal centre and
      // the transition ratio, which decide the move, carry no FP32 rounding
      const double* g = Wk.grad64 + ((size_t)buf * P.W * N + item) * 3 * P.S;
      const double* B = (prop ? A.binv64 : Wk.binv64) + boff;
      for (int l = s; l < n; l += 4) {
        const double b = B[(size_t)l * n];
        g0 += b * g[l];
        g1 += b * g[P.S + l];
        g2 += b * g[2 * P.S + l];
      }
    } else {
      const T* row = Wk.vgl + ((size_t)buf * P.W * N + item) * kComp * P.S;
      const T* B = (prop ? A.binv : Wk.binv) + boff;
      for (int l = s; l < n; l += 4) {
        const double b = (double)B[(size_t)l * n];
        g0 += b * (double)row[P.S + l];
        g1 += b * (double)row[2 * P.S + l];
        g2 += b * (double)row[3 * P.S + l];
      }
    }
    // Jastrow part: partners in three ranges (same spin, opposite spin, ions), every fourth
    const double xi0 = sx[i], xi1 = sy[i], xi2 = sz[i];
    const double L = P.L, invL = 1.0 / P.L;
    const bool up = i < P.n_up;
    auto range = [&](const Radial& R, int lo, int hi, bool ions) {
      for (int j = lo + s; j < hi; j += 4) {
        if (!ions && j == i) continue;
        double cx, cy, cz;
        if (ions) {
          const double* c = P.ions + 4 * (size_t)(j - lo);
          cx = c[0]; cy = c[1]; cz = c[2];
        } else {
          cx = sx[j]; cy = sy[j]; cz = sz[j];
        }
        const double dx = min_image(xi0 - cx, L, invL), dy = min_image(xi1 - cy, L, invL);
        const double dz = min_image(xi2 - cz, L, invL);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double ri = rsqrt(r2), r = r2 * ri;
        double u, du, d2u;
        radial_eval(R, r, u, du, d2u);
        const double f = du * ri;
        g0 += f * dx; g1 += f * dy; g2 += f * dz;
      }
    };
    range(up ? sj.same : sj.opp, 0, P.n_up, false);
    range(up ? sj.opp : sj.same, P.n_up, N, false);
    if (P.n_ions > 0 && sj.ei.kind != QMC_J_NONE) range(sj.ei, 0, P.n_ions, true);
    if (P.j3_on) {
      // three-body terms: grad_i u = u_a a^ + u_c c^ over ions near i and partners j near them
      const double h = P.j3_h;
      for (int I = 0; I < P.n_ions; ++I) {
        const double* ion = P.ions + 4 * (size_t)I;
        const double ax = min_image(xi0 - ion[0], L, invL), ay = min_image(xi1 - ion[1], L, invL);
        const double az = min_image(xi2 - ion[2], L, invL);
        const double a = sqrt(ax * ax + ay * ay + az * az);
        if (a >= h) continue;
        for (int j = s; j < N; j += 4) {
          if (j == i) continue;
          const double bx = min_image(sx[j] - ion[0], L, invL), by = min_image(sy[j] - ion[1], L, invL);
          const double bz = min_image(sz[j] - ion[2], L, invL);
          const double b = sqrt(bx * bx + by * by + bz * bz);
          if (b >= h) continue;
          const double cx = min_image(xi0 - sx[j], L, invL), cy = min_image(xi1 - sy[j], L, invL);
          const double cz = min_image(xi2 - sz[j], L, invL);
          const double c = sqrt(cx * cx + cy * cy + cz * cz);
          double d[6];
          u3_derivs(P, up == (j < P.n_up), a, b, c, d);
          const double fa = d[1] / a, fc = d[2] / c;
          g0 += fa * ax + fc * cx; g1 += fa * ay + fc * cy; g2 += fa * az + fc * cz;
        }
      }
    }
  }
  // the four slices of an electron are adjacent lanes
#pragma unroll
  for (int o = 1; o <= 2; o <<= 1) {
    g0 += __shfl_xor(g0, o, 64); g1 += __shfl_xor(g1, o, 64); g2 += __shfl_xor(g2, o, 64);
  }
  double tsum = 0.0;
  if (valid && s == 0) {
    double* vw = vel + ((size_t)w * N + i) * 3;
    vw[0] = g0; vw[1] = g1; vw[2] = g2;
    if (prop) {
      const uint32_t sweep = *Wk.sweep_ctr;
      const double tau = P.sigma * P.sigma;
      double a0, a1, b0, b1;
      uniform_pair(P, kPropose, 0, (uint32_t)w, sweep, (uint32_t)i, a0, a1);
      uniform_pair(P, kPropose, 1, (uint32_t)w, sweep, (uint32_t)i, b0, b1);
      const double ra = sqrt(-2.0 * log(1.0 - a0)), rb = sqrt(-2.0 * log(1.0 - b0));
      double sa, ca;
      sincos(2.0 * kPi * a1, &sa, &ca);
      const double cb = cos(2.0 * kPi * b1);
      const double sg[3] = {P.sigma * (ra * ca), P.sigma * (ra * sa), P.sigma * (rb * cb)};
      const double vn[3] = {g0, g1, g2};
      const double* vo = vcur + ((size_t)w * N + i) * 3;
      for (int a = 0; a < 3; ++a) {
        const double back = sg[a] + tau * (vo[a] + vn[a]);
        tsum += (sg[a] * sg[a] - back * back) / (2.0 * tau);
      }
    }
  }
  if (prop) {
    tsum = wave_sum_dpp(tsum);
    if (lane == 0) red[wave] = tsum;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) t += red[q];
      A.logT[(size_t)w * parts + p] = t;
    }
  }
}

// Decision and installation, one workgroup per walker.  u is the walker's uniform (the
// ACCEPT draw of electron 0, kept with electron 0's proposal); a singular matrix at R'
// rejects.  On acceptance the positions become the proposals, every electron's row buffer
// flag flips (the proposal rows become current), and the inverses, log|D| and signs become
// those of R'.  acc[w][i] = the decision for every electron, nacc[w] = N or 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ae_apply(SysParams P, Walkers<T> Wk, AeProposal<T> A) {
  __shared__ int sacc;
  const int w = blockIdx.x, tid = threadIdx.x;
  const int N = P.N;
  if (tid == 0) {
    const double u = Wk.prop[(size_t)w * N * 4 + 3];
    const double dlog = (A.logdet[2 * w] - Wk.logdet[2 * w]) + (A.logdet[2 * w + 1] - Wk.logdet[2 * w + 1]);
    double lt = 0.0;
    if (A.logT)
      for (int q = 0; q < A.logT_parts; ++q) lt += A.logT[(size_t)w * A.logT_parts + q];
    // fixed node: a move to where Psi has the other sign is rejected (the Jastrow factor is
    // positive, so the sign is that of D_up D_dn)
    const int crossed = A.fixed_node && A.status[w] == 0 &&
                        A.sign[2 * w] * A.sign[2 * w + 1] != Wk.sign[2 * w] * Wk.sign[2 * w + 1];
    if (A.crossed) A.crossed[w] = crossed;
    double dJ = 0.0;
    for (int q = 0; q < A.dj_parts; ++q) dJ += A.dj[(size_t)w * A.dj_parts + q];
    sacc = (A.status[w] == 0) && !crossed && (u < exp(2.0 * (dlog + dJ) + lt));
  }
  __syncthreads();
  const int acc = sacc;
  const size_t e0 = (size_t)w * N;
  for (int i = tid; i < N; i += kBlock) {
    Wk.acc[e0 + i] = (uint8_t)acc;
    if (acc) {
      const double* pr = Wk.prop + (e0 + i) * 4;
      double* p = Wk.pos + (e0 + i) * 3;
      p[0] = pr[0]; p[1] = pr[1]; p[2] = pr[2];
      Wk.cur[e0 + i] ^= (uint8_t)1;
    }
  }
  if (acc && A.vcur)   // the velocities at R' are those at the new current configuration
    for (int q = tid; q < 3 * N; q += kBlock) A.vcur[e0 * 3 + q] = A.vprop[e0 * 3 + q];
  if (acc) {
    // the walker's two inverses (bstride elements); as 16-byte vectors when every walker's
    // block starts on a 16-byte boundary (the buffers themselves are 256-byte aligned)
    const size_t base = (size_t)w * P.bstride;
    if (((size_t)P.bstride * sizeof(T)) % 16 == 0) {
      const size_t nv = (size_t)P.bstride * sizeof(T) / 16;
      const uint4* src = reinterpret_cast<const uint4*>(A.binv + base);
      uint4* dst = reinterpret_cast<uint4*>(Wk.binv + base);
      for (size_t q = tid; q < nv; q += kBlock) dst[q] = src[q];
    } else {
      for (size_t q = tid; q < (size_t)P.bstride; q += kBlock) Wk.binv[base + q] = A.binv[base + q];
    }
    if (A.binv64 && Wk.binv64)
      for (size_t q = tid; q < (size_t)P.bstride; q += kBlock) Wk.binv64[base + q] = A.binv64[base + q];
  }
  if (tid == 0) {
    if (acc) {
      Wk.logdet[2 * w] = A.logdet[2 * w];
      Wk.logdet[2 * w + 1] = A.logdet[2 * w + 1];
      Wk.sign[2 * w] = A.sign[2 * w];
      Wk.sign[2 * w + 1] = A.sign[2 * w + 1];
    }
    Wk.nacc[w] = acc ? (uint32_t)N : 0u;
    if (w == 0) *Wk.sweep_ctr += 1u;   // read by the next sweep's gather
  }
}

int jastrow_parts(int N) {
  const long pairs = (long)N * (N - 1) / 2;
  const long p = (pairs + 2047) / 2048;
  return (int)(p < 1 ? 1 : (p > 8 ? 8 : p));
}

hipError_t launch_ae_jastrow(const SysParams& P, const double* pos, const double* prop, double* dj,
                             int* status_prop, hipStream_t st) {
  if (P.W <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ae_jastrow, dim3((unsigned)P.W * jastrow_parts(P.N)), dim3(kBlock), 0, st, P, pos, prop,
                     dj, status_prop);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ae_velocity(const SysParams& P, const Walkers<T>& Wk, const AeProposal<T>& A, int prop,
                              double* vel, const double* vcur, hipStream_t st) {
  if (P.W <= 0) return hipSuccess;
  if (P.N > kVelMaxN) return hipErrorInvalidValue;
  if (prop && A.logT_parts != velocity_parts(P.N)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ae_velocity<T>, dim3((unsigned)P.W * velocity_parts(P.N)), dim3(kBlock), 0, st, P, Wk, A,
                     prop, vel, vcur);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ae_apply(const SysParams& P, const Walkers<T>& Wk, const AeProposal<T>& A, hipStream_t st) {
  if (P.W <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ae_apply<T>, dim3(P.W), dim3(kBlock), 0, st, P, Wk, A);
  return hipGetLastError();
}

template hipError_t launch_ae_velocity<float>(const SysParams&, const Walkers<float>&, const AeProposal<float>&,
                                              int, double*, const double*, hipStream_t);
template hipError_t launch_ae_velocity<double>(const SysParams&, const Walkers<double>&,
                                               const AeProposal<double>&, int, double*, const double*, hipStream_t);
template hipError_t launch_ae_apply<float>(const SysParams&, const Walkers<float>&, const AeProposal<float>&,
                                           hipStream_t);
template hipError_t launch_ae_apply<double>(const SysParams&, const Walkers<double>&,
                                            const AeProposal<double>&, hipStream_t);

}  // namespace qmc
