// k_chain.hip -- the sequential part of a particle-by-particle sweep.
//
// Section "Trial Moves": electrons are visited in order; electron i proposes
// r' (drawn by the gather kernel, whose orbital row v = phi(r') is already in
// HBM) and the move is accepted with probability min(1, |Psi'/Psi|^2), which
// for D_up D_dn exp(J) (equation eq:msdj) is R^2 exp(2 dJ) with
//   R  = sum_l v_l B[l][k]          (determinant ratio, B = A^-1, k = row of i)
//   dJ = sum_{j != i} [u2(|r'-r_j|) - u2(|r_i-r_j|)] + sum_I [u1(|r'-R_I|) - u1(|r_i-R_I|)]
// (section "Jastrow factors", minimum-image distances).  On acceptance the
// inverse gets the Sherman-Morrison rank-one update (section
// "Multi-Determinant Slater-Jastrow Form"):
//   B[l][m] -= B[l][k] (t_m - delta_mk) / R,   t_m = sum_j v_j B[j][m].
//
// One workgroup owns one walker for the whole sweep.  Positions, the spin
// block's proposals and buffer flags, small ion sets, and the active spin's
// inverse (whenever it fits) live in LDS.  The proposals' orbital rows do not
// depend on the chain's decisions, so they stream through a two-chunk LDS
// ring: the loads of chunk c+1 are issued when chunk c starts and have a whole
// chunk of moves to arrive, hiding the HBM latency.
#include <cstdlib>

#include "qmc_guard.hpp"
#include "qmc_kernels.hpp"

namespace qmc {

constexpr int kLdsIons = 256;     // ions staged in LDS up to this count

struct ChainLayout {
  size_t pos, prop, ions, red, vbuf, col, t, cur, acc, gx, gr, b, total;
};

__host__ __device__ inline ChainLayout chain_layout(int N, int nmax, int n_ions, int ldl, size_t ts,
                                                   bool b_in_lds, int rows_per_chunk) {
  ChainLayout L;
  size_t o = 0;
  L.pos = o; o += sizeof(double) * 3 * N;
  L.prop = o; o += sizeof(double) * 4 * nmax;
  L.ions = o; o += (n_ions <= kLdsIons) ? sizeof(double) * 4 * n_ions : 0;
  L.red = o; o += sizeof(double) * 9 * kWaves;
  o = (o + 15) & ~size_t(15);
  L.vbuf = o; o += ts * (size_t)2 * rows_per_chunk * nmax;
  o = (o + 15) & ~size_t(15);
  L.col = o; o += ts * nmax;
  o = (o + 15) & ~size_t(15);
  L.t = o; o += ts * nmax;
  o = (o + 15) & ~size_t(15);
  L.cur = o; o += nmax;
  L.acc = o; o += nmax;
  o = (o + 15) & ~size_t(15);
  L.gx = o; o += (ts == 4) ? sizeof(double) * nmax : 0;   // FP64 re-decision scratch (mixed)
  L.gr = o; o += (ts == 4) ? sizeof(double) * nmax : 0;
  L.b = o; o += b_in_lds ? ts * (size_t)nmax * ldl : 0;
  L.total = o;
  return L;
}

// Barrier between moves: LDS-only when the inverse lives in LDS (outstanding
// row loads stay in flight), a full barrier when the inverse is in global memory.
template <bool BLDS>
__device__ __forceinline__ void block_sync() {
  if (BLDS) sync_lds();
  else __syncthreads();
}

__device__ __forceinline__ double min_image_inv(double d, double L, double invL) {
  return d - L * rint(d * invL);
}

__device__ __forceinline__ double pair_u(const Jastrow& J, int kind, double r) {
  return kind == 0 ? radial_value(J.same, r) : (kind == 1 ? radial_value(J.opp, r) : radial_value(J.ei, r));
}

// VPT = orbital values per thread per row (n <= 256 * VPT); a chunk holds
// 16 / VPT rows, so the staging registers are always 16 values per thread.
template <typename T, bool BLDS, int VPT>
__global__ __launch_bounds__(kBlock) void k_chain(SysParams P, Walkers<T> Wk, int ldl) {
  constexpr int C = 16 / VPT;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Jastrow sj;
  const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = wave_of(tid);
  if (chain_skips(Wk, w)) return;
  const int N = P.N, nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  const ChainLayout lay = chain_layout(N, nmax, P.n_ions, ldl, sizeof(T), BLDS, C);
  double* spos = reinterpret_cast<double*>(smem + lay.pos);
  double* sprop = reinterpret_cast<double*>(smem + lay.prop);
  const bool ions_lds = P.n_ions <= kLdsIons;
  double* sion = reinterpret_cast<double*>(smem + lay.ions);
  const double* ions = ions_lds ? sion : P.ions;
  double* red = reinterpret_cast<double*>(smem + lay.red);
  T* vbuf = reinterpret_cast<T*>(smem + lay.vbuf);
  T* scol = reinterpret_cast<T*>(smem + lay.col);
  T* st = reinterpret_cast<T*>(smem + lay.t);
  uint8_t* scur = smem + lay.cur;
  uint8_t* sacc = smem + lay.acc;
  double* sgx = reinterpret_cast<double*>(smem + lay.gx);
  double* sgr = reinterpret_cast<double*>(smem + lay.gr);
  T* sB = reinterpret_cast<T*>(smem + lay.b);
  const double L = P.L, invL = 1.0 / P.L;

  {  // Jastrow parameters into LDS (indexed per lane below)
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.jas);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&sj);
    for (int q = tid; q < (int)(sizeof(Jastrow) / 4); q += kBlock) dst[q] = src[q];
  }
  for (int j = tid; j < 3 * N; j += kBlock) spos[j] = Wk.pos[(size_t)w * 3 * N + j];
  if (ions_lds)
    for (int j = tid; j < 4 * P.n_ions; j += kBlock) sion[j] = P.ions[j];
  uint32_t nacc = 0, nguard = 0;
  int parity = 0;

  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp ? P.n_dn : P.n_up;
    const int off = sp ? P.n_up : 0;
    if (n == 0) continue;
    const size_t item0 = (size_t)w * N + off;
    double logd = Wk.logdet[2 * w + sp];
    int sgn = Wk.sign[2 * w + sp];
    for (int q = tid; q < 4 * n; q += kBlock) sprop[q] = Wk.prop[item0 * 4 + q];
    for (int q = tid; q < n; q += kBlock) scur[q] = Wk.cur[item0 + q];
    T* Bg = Wk.binv + (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
    T* Bm;
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
    // mixed: the inverse error of B (its bound on ||v^T B|| is |v| ||B||_F)
    const double weta = sizeof(T) == 4 ? walker_eta(Wk, w, sp, n) : 0.0;
    const double bnorm = (sizeof(T) == 4 && Wk.eta) ? Wk.eta[4 * w + 2 + sp] : 0.0;
    // column split of the accept-path product t = v^T B: tpc threads per column
    int tpc = 1;
    while (tpc < 8 && tpc * 2 * n <= kBlock) tpc *= 2;

    // staging registers: this thread's elements of the next chunk's rows
    T stage[C][VPT];
    auto issue_chunk = [&](int c0) {
#pragma unroll
      for (int r = 0; r < C; ++r) {
        const int kk = c0 + r;
        if (kk < n) {
          const T* vrow = Wk.vgl + ((size_t)(1 - scur[kk]) * P.W * N + item0 + kk) * Wk.vstride;
#pragma unroll
          for (int c = 0; c < VPT; ++c) {
            const int j = tid + c * kBlock;
            stage[r][c] = (j < n) ? vrow[j] : T(0);
          }
        }
      }
    };
    issue_chunk(0);
    for (int k = 0; k < n; ++k) {
      const int i = off + k;
      const int kr = k % C;
      T* vrow_l = vbuf + ((size_t)((k / C) & 1) * C + kr) * nmax;   // this move's row in LDS
      if (kr == 0) {
        // the staged chunk goes to its LDS slot, then the next chunk's loads start
        T* slot = vbuf + (size_t)((k / C) & 1) * C * nmax;
#pragma unroll
        for (int r = 0; r < C; ++r)
#pragma unroll
          for (int c = 0; c < VPT; ++c) {
            const int j = tid + c * kBlock;
            if (j < n) slot[(size_t)r * nmax + j] = stage[r][c];
          }
        if (k + C < n) issue_chunk(k + C);
      }
      const double rx = sprop[4 * k], ry = sprop[4 * k + 1], rz = sprop[4 * k + 2], u = sprop[4 * k + 3];
      const double ec = sizeof(T) == 4 ? inverse_error_coef(Wk, w, i, N, weta) : 0.0;

      // determinant ratio (partial sums over this thread's own row elements)
      T rpart = T(0);
      double mpart = 0.0;   // mixed: sum |v_j B[j][k]|, the magnitude that bounds R's rounding
      double vpart = 0.0;   // mixed: |v|^2 (with ||B||_F it bounds ||v^T B||)
#pragma unroll
      for (int c = 0; c < VPT; ++c) {
        const int j = tid + c * kBlock;
        if (j < n) {
          const T vb = vrow_l[j] * Bm[(size_t)j * ldb + k];
          rpart += vb;
          if (sizeof(T) == 4) {
            mpart += fabs((double)vb);
            vpart += (double)vrow_l[j] * (double)vrow_l[j];
          }
        }
      }
      // Jastrow change (partial sums)
      const double xo = spos[3 * i], yo = spos[3 * i + 1], zo = spos[3 * i + 2];
      const bool up_i = i < P.n_up;
      double dj = 0.0;
      for (int j = tid; j < N + P.n_ions; j += kBlock) {
        if (j == i) continue;
        double cx, cy, cz;
        int kind;
        if (j < N) {
          cx = spos[3 * j]; cy = spos[3 * j + 1]; cz = spos[3 * j + 2];
          kind = ((j < P.n_up) == up_i) ? 0 : 1;
        } else {
          const double* ion = ions + 4 * (j - N);
          cx = ion[0]; cy = ion[1]; cz = ion[2];
          kind = 2;
        }
        double dx = min_image_inv(rx - cx, L, invL), dy = min_image_inv(ry - cy, L, invL);
        double dz = min_image_inv(rz - cz, L, invL);
        const double r1 = sqrt(dx * dx + dy * dy + dz * dz);
        dx = min_image_inv(xo - cx, L, invL); dy = min_image_inv(yo - cy, L, invL);
        dz = min_image_inv(zo - cz, L, invL);
        const double r0 = sqrt(dx * dx + dy * dy + dz * dz);
        dj += pair_u(sj, kind, r1) - pair_u(sj, kind, r0);
      }
      if (P.j3_on) {
        // three-body terms of electron i with partner j near ion I, at r' and at r
        const double h = P.j3_h;
        for (int q = tid; q < P.n_ions * N; q += kBlock) {
          const int I = q / N, j = q - I * N;
          if (j == i) continue;
          const double* ion = ions + 4 * I;
          auto d3 = [&](double x, double y, double z, double cx, double cy, double cz) {
            const double dx = min_image_inv(x - cx, L, invL), dy = min_image_inv(y - cy, L, invL);
            const double dz = min_image_inv(z - cz, L, invL);
            return sqrt(dx * dx + dy * dy + dz * dz);
          };
          const double a1 = d3(rx, ry, rz, ion[0], ion[1], ion[2]), a0 = d3(xo, yo, zo, ion[0], ion[1], ion[2]);
          if (a1 >= h && a0 >= h) continue;
          const double px = spos[3 * j], py = spos[3 * j + 1], pz = spos[3 * j + 2];
          const double b = d3(px, py, pz, ion[0], ion[1], ion[2]);
          if (b >= h) continue;
          const bool same = (j < P.n_up) == up_i;
          if (a1 < h) dj += u3_value(P, same, a1, b, d3(rx, ry, rz, px, py, pz));
          if (a0 < h) dj -= u3_value(P, same, a0, b, d3(xo, yo, zo, px, py, pz));
        }
      }
      // block reduction in a fixed order (bitwise repeatable)
      const double ra = wave_sum_dpp((double)rpart), rb = wave_sum_dpp(dj);
      const double rm = sizeof(T) == 4 ? wave_sum_dpp(mpart) : 0.0;
      const double rv = sizeof(T) == 4 ? wave_sum_dpp(vpart) : 0.0;
      double* rr = red + parity * 4 * kWaves;
      if (lane == 0) {
        rr[wave] = ra; rr[kWaves + wave] = rb; rr[2 * kWaves + wave] = rm; rr[3 * kWaves + wave] = rv;
      }
      block_sync<BLDS>();
      double Rd = 0.0, dJ = 0.0, Sm = 0.0, V2 = 0.0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) {
        Rd += rr[q]; dJ += rr[kWaves + q]; Sm += rr[2 * kWaves + q]; V2 += rr[3 * kWaves + q];
      }
      parity ^= 1;
      const T R = (T)Rd;
      const double ej = exp(2.0 * dJ);
      const double p32 = (double)R * (double)R * ej;
      double Rlog = (double)R;
      bool accept;
      // guard band: the relative tie guard widened by a bound on the FP32 rounding of R
      // (n + 1 unit roundoffs of the magnitude of its terms: heavy cancellation re-decides) and
      // by the error of the inverse itself, ||v^T B|| <= |v| ||B||_F times its measured residual
      const double band = sizeof(T) == 4
          ? P.tie_guard + 2.0 * (n + 1) * 5.9604644775390625e-08 * Sm / fabs((double)R) + 2.4e-7 +
                ec * sqrt(V2) * bnorm / fabs((double)R)
          : 0.0;
      if (sizeof(T) == 4 && fabs(u - p32) <= band * p32) {
        // near tie in FP32: decide again with an FP64 ratio (uniform branch)
        const double* v64 = Wk.val64 + ((size_t)(1 - scur[k]) * P.W * N + item0 + k) * P.S;
        Rlog = refined_ratio<T>(P, Wk, Bm, ldb, n, item0, scur, v64, k, sgx, sgr, red + 8 * kWaves, tid);
        accept = u < Rlog * Rlog * ej;
        ++nguard;
      } else {
        accept = u < p32;
      }

      if (accept) {
        for (int q = tid; q < n * tpc; q += kBlock) {
          const int m = q / tpc, part = q - m * tpc;
          T acc = T(0);
          for (int l = part; l < n; l += tpc) acc += vrow_l[l] * Bm[(size_t)l * ldb + m];
          for (int o = tpc >> 1; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
          if (part == 0) {
            st[m] = acc - (m == k ? T(1) : T(0));
            scol[m] = Bm[(size_t)m * ldb + k];
          }
        }
        block_sync<BLDS>();
        const T invR = T(1) / R;
        for (int l = wave; l < n; l += kWaves) {
          const T cl = scol[l] * invR;
          T* row = Bm + (size_t)l * ldb;
          for (int m = lane; m < n; m += 64) row[m] -= cl * st[m];
        }
        if (tid == 0) {
          spos[3 * i] = rx; spos[3 * i + 1] = ry; spos[3 * i + 2] = rz;
          scur[k] = (uint8_t)(1 - scur[k]);
          sacc[k] = 1;
        }
        ++nacc;
        logd += log(fabs(Rlog));
        if (Rlog < 0.0) sgn = -sgn;
        block_sync<BLDS>();
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
    if (BLDS) {
      for (int q = tid; q < n * n; q += kBlock) {
        const int l = q / n;
        Bg[q] = sB[l * ldl + (q - l * n)];
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < 3 * N; j += kBlock) Wk.pos[(size_t)w * 3 * N + j] = spos[j];
  if (tid == 0) {
    Wk.nacc[w] = nacc;
    Wk.nguard[w] += nguard;
    if (Wk.eta_age) Wk.eta_age[w] += 1u;
    if (Wk.fb && Wk.fb_sel == 1) Wk.pstat[2 * w + 1] += 1u;
    if (w == 0) *Wk.sweep_ctr += 1u;   // read by the next sweep's gather
  }
}

static int lds_budget() {
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

static int vpt_of(int nmax) { return nmax <= kBlock ? 1 : (nmax <= 2 * kBlock ? 2 : 4); }

size_t chain_lds_bytes(const SysParams& P, size_t tsize, bool b_in_lds) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  return chain_layout(P.N, nmax, P.n_ions, nmax | 1, tsize, b_in_lds, 16 / vpt_of(nmax)).total;
}

template <typename T, bool BLDS, int VPT>
static hipError_t launch_chain_variant(const SysParams& P, const Walkers<T>& Wk, hipStream_t st,
                                       size_t bytes, int ldl) {
  if (bytes > 65536) {
    const hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_chain<T, BLDS, VPT>));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_chain<T, BLDS, VPT>), dim3(P.W), dim3(kBlock), bytes, st, P, Wk, ldl);
  return hipGetLastError();
}

template <typename T, int VPT>
static hipError_t launch_chain_vpt(const SysParams& P, const Walkers<T>& Wk, hipStream_t st) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  const int ldl = nmax | 1;
  const size_t with_b = chain_layout(P.N, nmax, P.n_ions, ldl, sizeof(T), true, 16 / VPT).total;
  const size_t without_b = chain_layout(P.N, nmax, P.n_ions, ldl, sizeof(T), false, 16 / VPT).total;
  // QMC_CHAIN_GLOBAL_INVERSE=1 keeps the inverse in global memory even when it fits
  // LDS (lets the tests cover the large-system path on small systems).
  const char* fg = getenv("QMC_CHAIN_GLOBAL_INVERSE");
  const bool force_global = fg && fg[0] == '1';
  if (!force_global && with_b + sizeof(Jastrow) <= (size_t)lds_budget())
    return launch_chain_variant<T, true, VPT>(P, Wk, st, with_b, ldl);
  if (without_b + sizeof(Jastrow) > (size_t)lds_budget()) return hipErrorInvalidValue;
  return launch_chain_variant<T, false, VPT>(P, Wk, st, without_b, ldl);
}

template <typename T>
hipError_t launch_chain(const SysParams& P, const Walkers<T>& Wk, hipStream_t st) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  if (nmax > 4 * kBlock) return hipErrorInvalidValue;
  switch (vpt_of(nmax)) {
    case 1: return launch_chain_vpt<T, 1>(P, Wk, st);
    case 2: return launch_chain_vpt<T, 2>(P, Wk, st);
    default: return launch_chain_vpt<T, 4>(P, Wk, st);
  }
}

template hipError_t launch_chain<double>(const SysParams&, const Walkers<double>&, hipStream_t);
template hipError_t launch_chain<float>(const SysParams&, const Walkers<float>&, hipStream_t);

hipError_t chain_lds_limits() {
  const void* ks[] = {
      reinterpret_cast<const void*>(&k_chain<double, true, 1>), reinterpret_cast<const void*>(&k_chain<double, true, 2>),
      reinterpret_cast<const void*>(&k_chain<double, true, 4>), reinterpret_cast<const void*>(&k_chain<double, false, 1>),
      reinterpret_cast<const void*>(&k_chain<double, false, 2>), reinterpret_cast<const void*>(&k_chain<double, false, 4>),
      reinterpret_cast<const void*>(&k_chain<float, true, 1>), reinterpret_cast<const void*>(&k_chain<float, true, 2>),
      reinterpret_cast<const void*>(&k_chain<float, true, 4>), reinterpret_cast<const void*>(&k_chain<float, false, 1>),
      reinterpret_cast<const void*>(&k_chain<float, false, 2>), reinterpret_cast<const void*>(&k_chain<float, false, 4>)};
  for (const void* k : ks) {
    const hipError_t e = allow_dynamic_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qmc
