// k_measure.hip -- local energy of every walker after a sweep.
//
// Section "Hamiltonian": E_L = sum_n Psi^-1 H_n Psi, collected once all
// walkers have advanced one step.  For Psi = D_up D_dn exp(J):
//   T_L = -1/2 sum_i [ lap_i D / D + 2 grad_i ln D . grad_i J + lap_i J + |grad_i J|^2 ]
// with grad_i ln D = sum_l B[l][k] grad phi_l(r_i), lap_i D / D =
// sum_l B[l][k] lap phi_l(r_i) taken from the cached value/gradient/Laplacian
// row of each electron (no spline evaluation here), and the Jastrow
// derivatives summed over electron and ion partners (section "Jastrow
// factors").  The Coulomb terms (section "Long-Range Interactions") are Ewald
// sums: real-space pairs with erfc screening over the 27 nearest images, and
// a half-space reciprocal sum of |S(G)|^2 with the ions' S(G) precomputed.
#include "qmc_kernels.hpp"

namespace qmc {

__device__ __forceinline__ const Radial& pick(const Jastrow& J, int kind) {
  return kind == 0 ? J.same : (kind == 1 ? J.opp : J.ei);
}

// sum over the 27 images (d already minimum-imaged) of erfc(kappa r) / r, r < rcut
__device__ __forceinline__ double screened_images(double dx, double dy, double dz, double L,
                                                  double kappa, double rcut2) {
  double s = 0.0;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int c = -1; c <= 1; ++c) {
        const double x = dx + a * L, y = dy + b * L, z = dz + c * L;
        const double r2 = x * x + y * y + z * z;
        if (r2 < rcut2) {
          const double r = sqrt(r2);
          s += erfc(kappa * r) / r;
        }
      }
  return s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_measure(SysParams P, Walkers<T> Wk, EwaldParams E,
                                                    double* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Jastrow sj;
  __shared__ double red[3 * kWaves];
  const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = P.N;
  double* spos = reinterpret_cast<double*>(smem);
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.jas);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&sj);
    for (int q = tid; q < (int)(sizeof(Jastrow) / 4); q += kBlock) dst[q] = src[q];
  }
  for (int j = tid; j < 3 * N; j += kBlock) spos[j] = Wk.pos[(size_t)w * 3 * N + j];
  __syncthreads();

  double tkin = 0.0, vee = 0.0, vei = 0.0;
  const double rcut2 = E.rcut * E.rcut;
  for (int i = tid; i < N; i += kBlock) {
    const int sp = i < P.n_up ? 0 : 1;
    const int n = sp ? P.n_dn : P.n_up, k = i - (sp ? P.n_up : 0);
    const size_t item = (size_t)w * N + i;
    const T* row = Wk.vgl + ((size_t)Wk.cur[item] * P.W * N + item) * kComp * P.S;
    const T* B = Wk.binv + (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
    double gD[3] = {0.0, 0.0, 0.0}, lD = 0.0;
    for (int l = 0; l < n; ++l) {
      const double b = (double)B[(size_t)l * n + k];
      gD[0] += b * (double)row[P.S + l];
      gD[1] += b * (double)row[2 * P.S + l];
      gD[2] += b * (double)row[3 * P.S + l];
      lD += b * (double)row[4 * P.S + l];
    }
    const double xi = spos[3 * i], yi = spos[3 * i + 1], zi = spos[3 * i + 2];
    const bool up_i = i < P.n_up;
    double gJ[3] = {0.0, 0.0, 0.0}, lJ = 0.0, ee = 0.0, ei = 0.0;
    for (int j = 0; j < N + P.n_ions; ++j) {
      if (j == i) continue;
      double cx, cy, cz, q = 0.0;
      int kind;
      if (j < N) {
        cx = spos[3 * j]; cy = spos[3 * j + 1]; cz = spos[3 * j + 2];
        kind = ((j < P.n_up) == up_i) ? 0 : 1;
      } else {
        const double* ion = P.ions + 4 * (j - N);
        cx = ion[0]; cy = ion[1]; cz = ion[2]; q = ion[3];
        kind = 2;
      }
      const double dx = min_image(xi - cx, P.L), dy = min_image(yi - cy, P.L), dz = min_image(zi - cz, P.L);
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      double u, du, d2u;
      radial_eval(pick(sj, kind), r, u, du, d2u);
      const double f = du / r;
      gJ[0] += f * dx; gJ[1] += f * dy; gJ[2] += f * dz;
      lJ += d2u + 2.0 * f;
      if (E.enabled) {
        const double s = screened_images(dx, dy, dz, P.L, E.kappa, rcut2);
        if (j < N) ee += 0.5 * s;
        else ei -= q * s;
      }
    }
    const double dot = gD[0] * gJ[0] + gD[1] * gJ[1] + gD[2] * gJ[2];
    const double gJ2 = gJ[0] * gJ[0] + gJ[1] * gJ[1] + gJ[2] * gJ[2];
    tkin += -0.5 * (lD + 2.0 * dot + lJ + gJ2);
    vee += ee;
    vei += ei;
  }
  if (E.enabled) {
    for (int g = tid; g < E.n_g; g += kBlock) {
      const double Gx = E.gvec[4 * g], Gy = E.gvec[4 * g + 1], Gz = E.gvec[4 * g + 2], wg = E.gvec[4 * g + 3];
      double re = 0.0, im = 0.0;
      for (int i = 0; i < N; ++i) {
        double s, c;
        sincos(Gx * spos[3 * i] + Gy * spos[3 * i + 1] + Gz * spos[3 * i + 2], &s, &c);
        re -= c;   // electron charge -1
        im -= s;
      }
      vee += wg * (re * re + im * im);
      vei += wg * 2.0 * (re * E.s_ion[2 * g] + im * E.s_ion[2 * g + 1]);
    }
  }
  const double a = wave_sum(tkin), b = wave_sum(vee), c = wave_sum(vei);
  if (lane == 0) { red[wave] = a; red[kWaves + wave] = b; red[2 * kWaves + wave] = c; }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0, x = 0.0, y = 0.0;
    for (int q = 0; q < kWaves; ++q) { t += red[q]; x += red[kWaves + q]; y += red[2 * kWaves + q]; }
    out[4 * w + 0] = t;
    out[4 * w + 1] = E.enabled ? x + E.c_ee : 0.0;
    out[4 * w + 2] = E.enabled ? y + E.c_ei : 0.0;
    out[4 * w + 3] = E.enabled ? E.v_ii : 0.0;
  }
}

template <typename T>
hipError_t launch_measure(const SysParams& P, const Walkers<T>& Wk, const EwaldParams& E, double* out,
                          hipStream_t st) {
  const size_t bytes = sizeof(double) * 3 * (size_t)P.N;
  hipLaunchKernelGGL(k_measure<T>, dim3(P.W), dim3(kBlock), bytes, st, P, Wk, E, out);
  return hipGetLastError();
}

template hipError_t launch_measure<double>(const SysParams&, const Walkers<double>&, const EwaldParams&,
                                           double*, hipStream_t);
template hipError_t launch_measure<float>(const SysParams&, const Walkers<float>&, const EwaldParams&,
                                          double*, hipStream_t);

}  // namespace qmc
