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
// One workgroup owns one walker for the whole sweep; the walker's positions
// live in LDS, and so does the active spin's inverse whenever it fits.
#include "qmc_kernels.hpp"

namespace qmc {

template <typename T>
struct ChainLayout {
  // byte offsets inside the dynamic LDS block
  size_t pos, red, v, col, t, b, total;
};

template <typename T>
__host__ __device__ inline ChainLayout<T> chain_layout(int N, int nmax, int ldl, bool b_in_lds) {
  ChainLayout<T> L;
  size_t o = 0;
  L.pos = o; o += sizeof(double) * 3 * N;
  L.red = o; o += sizeof(double) * 4 * kWaves;
  o = (o + 15) & ~size_t(15);
  L.v = o; o += sizeof(T) * nmax;
  L.col = o; o += sizeof(T) * nmax;
  L.t = o; o += sizeof(T) * nmax;
  o = (o + 15) & ~size_t(15);
  L.b = o; o += b_in_lds ? sizeof(T) * (size_t)nmax * ldl : 0;
  L.total = o;
  return L;
}

__device__ __forceinline__ double pair_u(const Jastrow& J, int kind, double r) {
  return kind == 0 ? radial_value(J.same, r) : (kind == 1 ? radial_value(J.opp, r) : radial_value(J.ei, r));
}

template <typename T, bool BLDS>
__global__ __launch_bounds__(kBlock) void k_chain(SysParams P, Walkers<T> Wk, uint32_t sweep, int ldl) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Jastrow sj;
  const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = P.N, nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  const ChainLayout<T> lay = chain_layout<T>(N, nmax, ldl, BLDS);
  double* spos = reinterpret_cast<double*>(smem + lay.pos);
  double* red = reinterpret_cast<double*>(smem + lay.red);
  T* sv = reinterpret_cast<T*>(smem + lay.v);
  T* scol = reinterpret_cast<T*>(smem + lay.col);
  T* st = reinterpret_cast<T*>(smem + lay.t);
  T* sB = reinterpret_cast<T*>(smem + lay.b);

  {  // Jastrow parameters into LDS (indexed per lane below)
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.jas);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&sj);
    for (int q = tid; q < (int)(sizeof(Jastrow) / 4); q += kBlock) dst[q] = src[q];
  }
  for (int j = tid; j < 3 * N; j += kBlock) spos[j] = Wk.pos[(size_t)w * 3 * N + j];
  double logd[2] = {Wk.logdet[2 * w], Wk.logdet[2 * w + 1]};
  int sgn[2] = {Wk.sign[2 * w], Wk.sign[2 * w + 1]};
  uint32_t nacc = 0;
  int parity = 0;
  __syncthreads();

  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp ? P.n_dn : P.n_up;
    const int off = sp ? P.n_up : 0;
    if (n == 0) continue;
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
      __syncthreads();
    } else {
      Bm = Bg;
      ldb = n;
    }
    for (int k = 0; k < n; ++k) {
      const int i = off + k;
      const size_t item = (size_t)w * N + i;
      const double* pr = Wk.prop + item * 4;
      const double rx = pr[0], ry = pr[1], rz = pr[2], u = pr[3];
      const int cb = Wk.cur[item];
      const T* vrow = Wk.vgl + ((size_t)(1 - cb) * P.W * N + item) * kComp * P.S;

      // determinant ratio (partial sums) and orbital row into LDS
      T rpart = T(0);
      for (int j = tid; j < n; j += kBlock) {
        const T vj = vrow[j];
        sv[j] = vj;
        rpart += vj * Bm[(size_t)j * ldb + k];
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
          const double* ion = P.ions + 4 * (j - N);
          cx = ion[0]; cy = ion[1]; cz = ion[2];
          kind = 2;
        }
        double dx = min_image(rx - cx, P.L), dy = min_image(ry - cy, P.L), dz = min_image(rz - cz, P.L);
        const double r1 = sqrt(dx * dx + dy * dy + dz * dz);
        dx = min_image(xo - cx, P.L); dy = min_image(yo - cy, P.L); dz = min_image(zo - cz, P.L);
        const double r0 = sqrt(dx * dx + dy * dy + dz * dz);
        dj += pair_u(sj, kind, r1) - pair_u(sj, kind, r0);
      }
      // block reduction in a fixed order (bitwise repeatable)
      const double ra = wave_sum((double)rpart), rb = wave_sum(dj);
      double* rr = red + parity * 2 * kWaves;
      if (lane == 0) { rr[wave] = ra; rr[kWaves + wave] = rb; }
      __syncthreads();
      double Rd = 0.0, dJ = 0.0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) { Rd += rr[q]; dJ += rr[kWaves + q]; }
      parity ^= 1;
      const T R = (T)Rd;
      const bool accept = u < (double)R * (double)R * exp(2.0 * dJ);

      if (accept) {
        for (int m = tid; m < n; m += kBlock) {
          T acc = T(0);
          for (int l = 0; l < n; ++l) acc += sv[l] * Bm[(size_t)l * ldb + m];
          st[m] = acc - (m == k ? T(1) : T(0));
          scol[m] = Bm[(size_t)m * ldb + k];
        }
        __syncthreads();
        const T invR = T(1) / R;
        for (int l = tid / 64; l < n; l += kWaves) {
          const T cl = scol[l] * invR;
          T* row = Bm + (size_t)l * ldb;
          for (int m = lane; m < n; m += 64) row[m] -= cl * st[m];
        }
        if (tid == 0) {
          spos[3 * i] = rx; spos[3 * i + 1] = ry; spos[3 * i + 2] = rz;
          Wk.cur[item] = (uint8_t)(1 - cb);
          Wk.acc[item] = 1;
        }
        ++nacc;
        logd[sp] += log(fabs((double)R));
        if (R < T(0)) sgn[sp] = -sgn[sp];
        __syncthreads();
      } else if (tid == 0) {
        Wk.acc[item] = 0;
      }
    }
    if (BLDS) {
      for (int q = tid; q < n * n; q += kBlock) {
        const int l = q / n;
        Bg[q] = sB[l * ldl + (q - l * n)];
      }
      __syncthreads();
    }
  }
  for (int j = tid; j < 3 * N; j += kBlock) Wk.pos[(size_t)w * 3 * N + j] = spos[j];
  if (tid == 0) {
    Wk.logdet[2 * w] = logd[0];
    Wk.logdet[2 * w + 1] = logd[1];
    Wk.sign[2 * w] = sgn[0];
    Wk.sign[2 * w + 1] = sgn[1];
    Wk.nacc[w] = nacc;
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

size_t chain_lds_bytes(const SysParams& P, size_t tsize, bool b_in_lds) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  const int ldl = nmax | 1;
  if (tsize == sizeof(double)) return chain_layout<double>(P.N, nmax, ldl, b_in_lds).total;
  return chain_layout<float>(P.N, nmax, ldl, b_in_lds).total;
}

template <typename T>
hipError_t launch_chain(const SysParams& P, const Walkers<T>& Wk, uint32_t sweep, hipStream_t st) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  const int ldl = nmax | 1;
  const size_t with_b = chain_layout<T>(P.N, nmax, ldl, true).total + sizeof(Jastrow);
  if (with_b <= (size_t)lds_budget()) {
    const size_t bytes = chain_layout<T>(P.N, nmax, ldl, true).total;
    if (bytes > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chain<T, true>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_chain<T, true>), dim3(P.W), dim3(kBlock), bytes, st, P, Wk, sweep, ldl);
  } else {
    const size_t bytes = chain_layout<T>(P.N, nmax, ldl, false).total;
    hipLaunchKernelGGL((k_chain<T, false>), dim3(P.W), dim3(kBlock), bytes, st, P, Wk, sweep, ldl);
  }
  return hipGetLastError();
}

template hipError_t launch_chain<double>(const SysParams&, const Walkers<double>&, uint32_t, hipStream_t);
template hipError_t launch_chain<float>(const SysParams&, const Walkers<float>&, uint32_t, hipStream_t);

}  // namespace qmc
