// k_drift.hip -- particle-by-particle drift-diffusion sweeps (section "Trial Moves": one
// electron's move drawn from the transition probability with the wavefunction force
// F = 2 grad ln Psi and lambda = 1/2, time step tau = sigma^2, accepted by eq.
// accept_reject with the ratio of the transition probabilities).
//
// Electron i's proposal r' = r_i + tau v + sigma xi is centred on its velocity
// v = grad_i ln|Psi| at the configuration the earlier moves of the sweep left, so unlike the
// plain sweep the proposals cannot be gathered for the whole sweep ahead of the chain: each
// move evaluates its own orbital row at r' inside the chain.  Per move, one workgroup (one
// walker) computes
//   v   = sum_l grad phi_l(r_i) B[l][k] + grad_i J        (current row, current inverse)
//   r'  = r_i + tau v + sigma xi                           (the sweep's PROPOSE draws)
//   the value, gradient and Laplacian of every orbital of the spin block at r' (each wave one
//   x-slab of the 4x4x4 stencil, its lanes along the orbitals; the slabs added in order),
//   written to the row buffer that does not hold the current row (as the gather would)
//   R   = sum_l phi_l(r') B[l][k],  dJ,  grad_i J at r'
//   v'  = sum_l grad phi_l(r') B[l][k] / R + grad_i J(R') (B[:,k] / R is the updated column)
//   ln T(r'->r)/T(r->r') = [|sigma xi|^2 - |sigma xi + tau (v + v')|^2] / (2 tau)
// and accepts iff u < R^2 exp(2 dJ + ln T ratio); R = 0 rejects, and with fixed_node so does
// R < 0 (a change of the sign of Psi).  Accepted moves update the inverse by
// Sherman-Morrison as in the plain chain.  FP64 throughout.
#include <cstdlib>

#include "qmc_kernels.hpp"

namespace qmc {

namespace {

constexpr int kDriftIons = 256;   // ions staged in LDS up to this count

struct DriftLayout {
  size_t pos, ions, red, part, row, col, t, cur, acc, b, total;
};

__host__ __device__ inline DriftLayout drift_layout(int N, int nmax, int n_ions, int ldl, bool b_in_lds) {
  DriftLayout L;
  size_t o = 0;
  L.pos = o; o += sizeof(double) * 3 * N;
  L.ions = o; o += n_ions <= kDriftIons ? sizeof(double) * 4 * n_ions : 0;
  L.red = o; o += sizeof(double) * 2 * 8 * kWaves;
  o = (o + 15) & ~size_t(15);
  L.part = o; o += sizeof(double) * (size_t)kWaves * kComp * nmax;   // each wave's slab sums
  L.row = o; o += sizeof(double) * (size_t)kComp * nmax;             // the proposal's row
  L.col = o; o += sizeof(double) * nmax;
  L.t = o; o += sizeof(double) * nmax;
  L.cur = o; o += nmax;
  L.acc = o; o += nmax;
  o = (o + 15) & ~size_t(15);
  L.b = o; o += b_in_lds ? sizeof(double) * (size_t)nmax * ldl : 0;
  L.total = o;
  return L;
}

template <bool BLDS>
__device__ __forceinline__ void drift_sync() {
  if (BLDS) sync_lds();
  else __syncthreads();
}

// Sum of v over the workgroup into slot q of buf (kWaves partials), no barrier.
__device__ __forceinline__ void wave_partial(double v, double* buf, int q, int lane, int wave) {
  v = wave_sum_dpp(v);
  if (lane == 0) buf[q * kWaves + wave] = v;
}

// Entry a of a four-entry array without indexing it dynamically (a is wave-uniform; an
// indexed private array would live in scratch memory).
template <typename V>
__device__ __forceinline__ V pick4(const V (&x)[4], int a) {
  return a == 0 ? x[0] : (a == 1 ? x[1] : (a == 2 ? x[2] : x[3]));
}

__device__ __forceinline__ double partial_total(const double* buf, int q) {
  double s = 0.0;
#pragma unroll
  for (int p = 0; p < kWaves; ++p) s += buf[q * kWaves + p];
  return s;
}

}  // namespace

// One workgroup per walker, the whole sweep (both spin blocks in turn).  sweep: the index of
// this sweep in the random streams; crossed (nullable): [W] node-crossing rejections of the
// sweep (fixed_node).
template <bool BLDS>
__global__ __launch_bounds__(kBlock) void k_chain_drift(SysParams P, Walkers<double> Wk,
                                                        const double* __restrict__ table, int ldl,
                                                        uint32_t sweep, int fixed_node, int* crossed) {
  static_assert(kWaves == 4, "one wave per x-slab of the 4x4x4 stencil");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Jastrow sj;
  const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = P.N, nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  const DriftLayout lay = drift_layout(N, nmax, P.n_ions, ldl, BLDS);
  double* spos = reinterpret_cast<double*>(smem + lay.pos);
  const bool ions_lds = P.n_ions <= kDriftIons;
  double* sion = reinterpret_cast<double*>(smem + lay.ions);
  const double* ions = ions_lds ? sion : P.ions;
  double* redA = reinterpret_cast<double*>(smem + lay.red);   // velocity sums
  double* redD = redA + 8 * kWaves;                           // ratio, gradients, Jastrow sums
  double* spart = reinterpret_cast<double*>(smem + lay.part);
  double* srow = reinterpret_cast<double*>(smem + lay.row);
  double* scol = reinterpret_cast<double*>(smem + lay.col);
  double* st = reinterpret_cast<double*>(smem + lay.t);
  uint8_t* scur = smem + lay.cur;
  uint8_t* sacc = smem + lay.acc;
  double* sB = reinterpret_cast<double*>(smem + lay.b);
  const double L = P.L, invL = 1.0 / P.L;
  const double tau = P.sigma * P.sigma;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.jas);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&sj);
    for (int q = tid; q < (int)(sizeof(Jastrow) / 4); q += kBlock) dst[q] = src[q];
  }
  for (int j = tid; j < 3 * N; j += kBlock) spos[j] = Wk.pos[(size_t)w * 3 * N + j];
  if (ions_lds)
    for (int j = tid; j < 4 * P.n_ions; j += kBlock) sion[j] = P.ions[j];
  uint32_t nacc = 0;
  int ncross = 0;

  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp ? P.n_dn : P.n_up;
    const int off = sp ? P.n_up : 0;
    if (n == 0) continue;
    const size_t item0 = (size_t)w * N + off;
    double logd = Wk.logdet[2 * w + sp];
    int sgn = Wk.sign[2 * w + sp];
    for (int q = tid; q < n; q += kBlock) scur[q] = Wk.cur[item0 + q];
    double* Bg = Wk.binv + (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
    double* Bm;
    int ldb;
    if (BLDS) {
      for (int q = tid; q < n * n; q += kBlock) {
        const int l = q / n;
        sB[l * ldl + (q - l * n)] = Bg[q];
      }
      Bm = sB;
      ldb = ldl;
    } else {
      Bm = Bg;
      ldb = n;
    }
    __syncthreads();
    int tpc = 1;   // threads per column of the accept-path product t = v^T B
    while (tpc < 8 && tpc * 2 * n <= kBlock) tpc *= 2;

    for (int k = 0; k < n; ++k) {
      const int i = off + k;
      const bool up_i = i < P.n_up;
      const double xo = spos[3 * i], yo = spos[3 * i + 1], zo = spos[3 * i + 2];
      // (1) v at the current configuration: determinant part from the current row and the
      // current inverse column, Jastrow part over every partner
      {
        const double* grow = Wk.vgl + ((size_t)scur[k] * P.W * N + item0 + k) * kComp * P.S;
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, h0 = 0.0, h1 = 0.0, h2 = 0.0;
        for (int l = tid; l < n; l += kBlock) {
          const double b = Bm[(size_t)l * ldb + k];
          g0 += b * grow[P.S + l];
          g1 += b * grow[2 * P.S + l];
          g2 += b * grow[3 * P.S + l];
        }
        for (int j = tid; j < N + P.n_ions; j += kBlock) {
          if (j == i) continue;
          double cx, cy, cz;
          const Radial* R;
          if (j < N) {
            cx = spos[3 * j]; cy = spos[3 * j + 1]; cz = spos[3 * j + 2];
            R = ((j < P.n_up) == up_i) ? &sj.same : &sj.opp;
          } else {
            const double* ion = ions + 4 * (j - N);
            cx = ion[0]; cy = ion[1]; cz = ion[2];
            R = &sj.ei;
          }
          const double dx = min_image(xo - cx, L, invL), dy = min_image(yo - cy, L, invL);
          const double dz = min_image(zo - cz, L, invL);
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          double u, du, d2u;
          radial_eval(*R, r, u, du, d2u);
          const double f = du / r;
          h0 += f * dx; h1 += f * dy; h2 += f * dz;
        }
        if (P.j3_on) {
          const double hc = P.j3_h;
          for (int q = tid; q < P.n_ions * N; q += kBlock) {
            const int I = q / N, j = q - I * N;
            if (j == i) continue;
            const double* ion = ions + 4 * I;
            const double ax = min_image(xo - ion[0], L, invL), ay = min_image(yo - ion[1], L, invL);
            const double az = min_image(zo - ion[2], L, invL);
            const double a = sqrt(ax * ax + ay * ay + az * az);
            if (a >= hc) continue;
            const double bx = min_image(spos[3 * j] - ion[0], L, invL);
            const double by = min_image(spos[3 * j + 1] - ion[1], L, invL);
            const double bz = min_image(spos[3 * j + 2] - ion[2], L, invL);
            const double b = sqrt(bx * bx + by * by + bz * bz);
            if (b >= hc) continue;
            const double cx = min_image(xo - spos[3 * j], L, invL), cy = min_image(yo - spos[3 * j + 1], L, invL);
            const double cz = min_image(zo - spos[3 * j + 2], L, invL);
            const double c = sqrt(cx * cx + cy * cy + cz * cz);
            double d[6];
            u3_derivs(P, up_i == (j < P.n_up), a, b, c, d);
            const double fa = d[1] / a, fc = d[2] / c;
            h0 += fa * ax + fc * cx; h1 += fa * ay + fc * cy; h2 += fa * az + fc * cz;
          }
        }
        wave_partial(g0 + h0, redA, 0, lane, wave);
        wave_partial(g1 + h1, redA, 1, lane, wave);
        wave_partial(g2 + h2, redA, 2, lane, wave);
      }
      drift_sync<BLDS>();
      const double v0 = partial_total(redA, 0), v1 = partial_total(redA, 1), v2 = partial_total(redA, 2);
      // (2) the proposal and the uniform (the same counters as the plain sweep's gather)
      double a0, a1, b0, b1, u, unused;
      uniform_pair(P, kPropose, 0, (uint32_t)w, sweep, (uint32_t)i, a0, a1);
      uniform_pair(P, kPropose, 1, (uint32_t)w, sweep, (uint32_t)i, b0, b1);
      uniform_pair(P, kAccept, 0, (uint32_t)w, sweep, (uint32_t)i, u, unused);
      const double ra = sqrt(-2.0 * log(1.0 - a0)), rb = sqrt(-2.0 * log(1.0 - b0));
      double sa, ca;
      sincos(2.0 * kPi * a1, &sa, &ca);
      const double sx0 = P.sigma * (ra * ca), sx1 = P.sigma * (ra * sa), sx2 = P.sigma * (rb * cos(2.0 * kPi * b1));
      const double rx = wrap_cell(xo + tau * v0 + sx0, L), ry = wrap_cell(yo + tau * v1 + sx1, L);
      const double rz = wrap_cell(zo + tau * v2 + sx2, L);
      // (3) the orbital row at r': wave a takes x-slab a, lanes the orbitals
      {
        Axis ax, ay, az;
        axis_weights(rx, L, P.gx, ax);
        axis_weights(ry, L, P.gy, ay);
        axis_weights(rz, L, P.gz, az);
        const int a = wave;
        const size_t xbase = (size_t)pick4(ax.idx, a) * P.gy;
        const double xw = pick4(ax.w, a), xd = pick4(ax.dw, a), xdd = pick4(ax.d2w, a);
        double* part = spart + (size_t)a * kComp * nmax;
#pragma unroll 1
        for (int l = lane; l < n; l += 64) {
          double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0, c4 = 0.0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const double* zrow = table + ((xbase + ay.idx[b]) * P.gz) * (size_t)P.S + l;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const double coef = zrow[(size_t)az.idx[c] * P.S];
              const double wyz = ay.w[b] * az.w[c];
              c0 += xw * wyz * coef;
              c1 += xd * wyz * coef;
              c2 += xw * ay.dw[b] * az.w[c] * coef;
              c3 += xw * ay.w[b] * az.dw[c] * coef;
              c4 += (xdd * wyz + xw * ay.d2w[b] * az.w[c] + xw * ay.w[b] * az.d2w[c]) * coef;
            }
          }
          part[l] = c0;
          part[nmax + l] = c1;
          part[2 * nmax + l] = c2;
          part[3 * nmax + l] = c3;
          part[4 * nmax + l] = c4;
        }
      }
      sync_lds();
      {
        double* vout = Wk.vgl + ((size_t)(1 - scur[k]) * P.W * N + item0 + k) * kComp * P.S;
        const size_t ps = (size_t)kComp * nmax;
        for (int q = tid; q < kComp * n; q += kBlock) {
          const int c = q / n, l = q - c * n;
          const size_t o = (size_t)c * nmax + l;
          const double s = ((spart[o] + spart[ps + o]) + spart[2 * ps + o]) + spart[3 * ps + o];
          srow[o] = s;
          vout[(size_t)c * P.S + l] = s;
        }
      }
      sync_lds();
      // (4) ratio, determinant gradient at r', Jastrow change and gradient at r'
      {
        double pr = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
        for (int l = tid; l < n; l += kBlock) {
          const double b = Bm[(size_t)l * ldb + k];
          pr += srow[l] * b;
          g0 += srow[nmax + l] * b;
          g1 += srow[2 * nmax + l] * b;
          g2 += srow[3 * nmax + l] * b;
        }
        double dj = 0.0, h0 = 0.0, h1 = 0.0, h2 = 0.0;
        for (int j = tid; j < N + P.n_ions; j += kBlock) {
          if (j == i) continue;
          double cx, cy, cz;
          const Radial* R;
          if (j < N) {
            cx = spos[3 * j]; cy = spos[3 * j + 1]; cz = spos[3 * j + 2];
            R = ((j < P.n_up) == up_i) ? &sj.same : &sj.opp;
          } else {
            const double* ion = ions + 4 * (j - N);
            cx = ion[0]; cy = ion[1]; cz = ion[2];
            R = &sj.ei;
          }
          double dx = min_image(rx - cx, L, invL), dy = min_image(ry - cy, L, invL);
          double dz = min_image(rz - cz, L, invL);
          const double r1 = sqrt(dx * dx + dy * dy + dz * dz);
          double u1, du1, d2u1;
          radial_eval(*R, r1, u1, du1, d2u1);
          const double f = du1 / r1;
          h0 += f * dx; h1 += f * dy; h2 += f * dz;
          dx = min_image(xo - cx, L, invL); dy = min_image(yo - cy, L, invL); dz = min_image(zo - cz, L, invL);
          dj += u1 - radial_value(*R, sqrt(dx * dx + dy * dy + dz * dz));
        }
        if (P.j3_on) {
          const double hc = P.j3_h;
          for (int q = tid; q < P.n_ions * N; q += kBlock) {
            const int I = q / N, j = q - I * N;
            if (j == i) continue;
            const double* ion = ions + 4 * I;
            const double ax = min_image(rx - ion[0], L, invL), ay = min_image(ry - ion[1], L, invL);
            const double az = min_image(rz - ion[2], L, invL);
            const double a1 = sqrt(ax * ax + ay * ay + az * az);
            double ex = min_image(xo - ion[0], L, invL), ey = min_image(yo - ion[1], L, invL);
            double ez = min_image(zo - ion[2], L, invL);
            const double a0 = sqrt(ex * ex + ey * ey + ez * ez);
            if (a1 >= hc && a0 >= hc) continue;
            const double px = spos[3 * j], py = spos[3 * j + 1], pz = spos[3 * j + 2];
            const double bx = min_image(px - ion[0], L, invL), by = min_image(py - ion[1], L, invL);
            const double bz = min_image(pz - ion[2], L, invL);
            const double b = sqrt(bx * bx + by * by + bz * bz);
            if (b >= hc) continue;
            const bool same = (j < P.n_up) == up_i;
            if (a1 < hc) {
              const double cx = min_image(rx - px, L, invL), cy = min_image(ry - py, L, invL);
              const double cz = min_image(rz - pz, L, invL);
              const double c = sqrt(cx * cx + cy * cy + cz * cz);
              double d[6];
              u3_derivs(P, same, a1, b, c, d);
              dj += d[0];
              const double fa = d[1] / a1, fc = d[2] / c;
              h0 += fa * ax + fc * cx; h1 += fa * ay + fc * cy; h2 += fa * az + fc * cz;
            }
            if (a0 < hc) {
              ex = min_image(xo - px, L, invL); ey = min_image(yo - py, L, invL); ez = min_image(zo - pz, L, invL);
              dj -= u3_value(P, same, a0, b, sqrt(ex * ex + ey * ey + ez * ez));
            }
          }
        }
        wave_partial(pr, redD, 0, lane, wave);
        wave_partial(g0, redD, 1, lane, wave);
        wave_partial(g1, redD, 2, lane, wave);
        wave_partial(g2, redD, 3, lane, wave);
        wave_partial(dj, redD, 4, lane, wave);
        wave_partial(h0, redD, 5, lane, wave);
        wave_partial(h1, redD, 6, lane, wave);
        wave_partial(h2, redD, 7, lane, wave);
      }
      drift_sync<BLDS>();
      const double R = partial_total(redD, 0), dJ = partial_total(redD, 4);
      // (5) the decision (uniform across the workgroup)
      const bool cross = fixed_node && R < 0.0;
      bool accept = false;
      if (R != 0.0 && !cross) {
        const double iR = 1.0 / R;
        const double vp0 = partial_total(redD, 1) * iR + partial_total(redD, 5);
        const double vp1 = partial_total(redD, 2) * iR + partial_total(redD, 6);
        const double vp2 = partial_total(redD, 3) * iR + partial_total(redD, 7);
        const double k0 = sx0 + tau * (v0 + vp0), k1 = sx1 + tau * (v1 + vp1), k2 = sx2 + tau * (v2 + vp2);
        const double lt = ((sx0 * sx0 - k0 * k0) + (sx1 * sx1 - k1 * k1) + (sx2 * sx2 - k2 * k2)) / (2.0 * tau);
        accept = u < R * R * exp(2.0 * dJ + lt);
      }
      ncross += cross ? 1 : 0;
      if (accept) {
        for (int q = tid; q < n * tpc; q += kBlock) {
          const int m = q / tpc, part = q - m * tpc;
          double acc = 0.0;
          for (int l = part; l < n; l += tpc) acc += srow[l] * Bm[(size_t)l * ldb + m];
          for (int o = tpc >> 1; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
          if (part == 0) {
            st[m] = acc - (m == k ? 1.0 : 0.0);
            scol[m] = Bm[(size_t)m * ldb + k];
          }
        }
        drift_sync<BLDS>();
        const double invR = 1.0 / R;
        for (int l = wave; l < n; l += kWaves) {
          const double cl = scol[l] * invR;
          double* row = Bm + (size_t)l * ldb;
          for (int m = lane; m < n; m += 64) row[m] -= cl * st[m];
        }
        if (tid == 0) {
          spos[3 * i] = rx; spos[3 * i + 1] = ry; spos[3 * i + 2] = rz;
          scur[k] = (uint8_t)(1 - scur[k]);
          sacc[k] = 1;
        }
        ++nacc;
        logd += log(fabs(R));
        if (R < 0.0) sgn = -sgn;
        drift_sync<BLDS>();
      } else if (tid == 0) {
        sacc[k] = 0;
      }
    }
    __syncthreads();
    for (int q = tid; q < n; q += kBlock) {
      Wk.cur[item0 + q] = scur[q];
      Wk.acc[item0 + q] = sacc[q];
    }
    if (tid == 0) {
      Wk.logdet[2 * w + sp] = logd;
      Wk.sign[2 * w + sp] = sgn;
    }
    if (BLDS)
      for (int q = tid; q < n * n; q += kBlock) {
        const int l = q / n;
        Bg[q] = sB[l * ldl + (q - l * n)];
      }
    __syncthreads();
  }
  for (int j = tid; j < 3 * N; j += kBlock) Wk.pos[(size_t)w * 3 * N + j] = spos[j];
  if (tid == 0) {
    Wk.nacc[w] = nacc;
    if (crossed) crossed[w] = ncross;
    if (w == 0) *Wk.sweep_ctr += 1u;   // kept equal to the sweeps run
  }
}

namespace {

int drift_lds_budget() {
  static int budget = -1;
  if (budget < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      budget = v;
    else
      budget = 65536;
  }
  return budget;
}

}  // namespace

hipError_t launch_chain_drift(const SysParams& P, const Walkers<double>& Wk, const double* table, uint32_t sweep,
                              int fixed_node, int* crossed, hipStream_t st) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  const int ldl = nmax | 1;
  const size_t with_b = drift_layout(P.N, nmax, P.n_ions, ldl, true).total;
  const size_t without_b = drift_layout(P.N, nmax, P.n_ions, ldl, false).total;
  const size_t budget = (size_t)drift_lds_budget() - sizeof(Jastrow);
  // QMC_CHAIN_GLOBAL_INVERSE=1 keeps the inverse in global memory even when it fits LDS
  const char* fg = getenv("QMC_CHAIN_GLOBAL_INVERSE");
  const bool force_global = fg && fg[0] == '1';
  if (!force_global && with_b <= budget) {
    hipLaunchKernelGGL(k_chain_drift<true>, dim3(P.W), dim3(kBlock), with_b, st, P, Wk, table, ldl, sweep,
                       fixed_node, crossed);
    return hipGetLastError();
  }
  if (without_b > budget) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chain_drift<false>, dim3(P.W), dim3(kBlock), without_b, st, P, Wk, table, ldl, sweep,
                     fixed_node, crossed);
  return hipGetLastError();
}

bool drift_chain_fits(const SysParams& P) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  return drift_layout(P.N, nmax, P.n_ions, nmax | 1, false).total + sizeof(Jastrow) <= (size_t)drift_lds_budget();
}

hipError_t drift_lds_limits() {
  const void* ks[] = {reinterpret_cast<const void*>(&k_chain_drift<true>),
                      reinterpret_cast<const void*>(&k_chain_drift<false>)};
  for (const void* k : ks) {
    const hipError_t e = allow_dynamic_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qmc
