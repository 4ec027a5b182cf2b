// k_measure.hip -- local energy of every walker after a sweep.
//
// Section "Hamiltonian": E_L = sum_n Psi^-1 H_n Psi, collected once all
// walkers have advanced one step.  For Psi = D_up D_dn exp(J):
//   T_L = -1/2 sum_i [ lap_i D / D + 2 grad_i ln D . grad_i J + lap_i J + |grad_i J|^2 ]
// with grad_i ln D = sum_l B[l][k] grad phi_l(r_i) and lap_i D / D =
// sum_l B[l][k] lap phi_l(r_i) taken from each electron's cached
// value/gradient/Laplacian row (no spline evaluation here), and the Jastrow
// derivatives summed over electron and ion partners (section "Jastrow
// factors").  The Coulomb terms (section "Long-Range Interactions") are Ewald
// sums with splitting kappa: erfc-screened pairs over every image closer than
// the cutoff (one cell side), and the half-space reciprocal sum
// sum_G w(G) |S(G)|^2 with S(G) built segment by segment along Gz: one sincos
// per (segment, electron) and a complex recurrence for the next Gz.
//
// Several workgroups per walker (see measure_part); every phase spreads over
// all threads and combines partial sums in a fixed order (bitwise repeatable).
#include "qmc_kernels.hpp"

namespace qmc {

constexpr int kSeg = kEwaldSeg;

__device__ __forceinline__ const Radial& pick(const Jastrow& J, int kind) {
  return kind == 0 ? J.same : (kind == 1 ? J.opp : J.ei);
}

// In LDS the tables are stored coefficient-major, c_m of interval i at [m][i]: the lanes of
// a wave look up unrelated intervals, and with consecutive intervals in consecutive banks
// their reads spread over all banks (interval-major rows of 8 doubles would put every
// lane's c_m in one of a few banks).
constexpr int kTabInt = kHInt + kGInt;

// erfc(kappa r) / r = 1 / r - kappa H(kappa^2 r^2) for r^2 < rcut^2, H from its table.
__device__ __forceinline__ double screened(double r2, double kappa, const double* __restrict__ htab) {
  const double ri = rsqrt(r2);
  const double x = kappa * kappa * r2;
  const int i = min((int)(x * (1.0 / kHW)), kHInt - 1);
  const double u = (x - (i + 0.5) * kHW) * (2.0 / kHW);
  const double* c = htab + i;
  double h = c[kHDeg * kTabInt];
#pragma unroll
  for (int m = kHDeg - 1; m >= 0; --m) h = h * u + c[m * kTabInt];
  return ri - kappa * h;
}

// G(x) = erfc(sqrt x) / sqrt x from its table, for kGX0 <= x < 5.5^2.
__device__ __forceinline__ double screened_tail(double x, const double* __restrict__ htab) {
  const int i = max(0, min((int)((x - kGX0) * (1.0 / kHW)), kGInt - 1));
  const double u = (x - (kGX0 + (i + 0.5) * kHW)) * (2.0 / kHW);
  const double* c = htab + kHInt + i;
  double g = c[kHDeg * kTabInt];
#pragma unroll
  for (int m = kHDeg - 1; m >= 0; --m) g = g * u + c[m * kTabInt];
  return g;
}

// sum of erfc(kappa r) / r over the images of d (minimum-imaged) with r < rcut <= L:
// per axis only the shift toward the nearer neighbouring cell can qualify.  The
// minimum image itself is always inside the cutoff (r <= sqrt(3) L / 2); the others lie
// at r >= L / 2 and take the erfc table.
__device__ __forceinline__ double screened_images(double dx, double dy, double dz, double L,
                                                  double kappa, double rcut2, const double* htab) {
  const double sx = dx > 0.0 ? -L : L, sy = dy > 0.0 ? -L : L, sz = dz > 0.0 ? -L : L;
  const double k2 = kappa * kappa;
  double s = screened(dx * dx + dy * dy + dz * dz, kappa, htab);
#pragma unroll
  for (int m = 1; m < 8; ++m) {
    const double x = dx + ((m & 1) ? sx : 0.0);
    const double y = dy + ((m & 2) ? sy : 0.0);
    const double z = dz + ((m & 4) ? sz : 0.0);
    const double r2 = x * x + y * y + z * z;
    if (r2 < rcut2) s += kappa * screened_tail(k2 * r2, htab);
  }
  return s;
}

struct MeasureLayout {
  size_t pos, ez, gd, ld, gjp, ljp, htab, total;
  int nloc;    // electrons per part (upper bound)
  int parts;   // Jastrow partner split per electron
};

// Every walker's local energy is computed by np workgroups (parts): part p
// takes the kinetic terms of electrons p nloc .. (p + 1) nloc - 1, the p-th
// contiguous block of the electron pairs and of the electron-ion pairs, and
// every np-th reciprocal segment; it writes five partial sums, and a second
// kernel adds the parts of a walker in a fixed order.  Spreading a walker
// over several workgroups keeps enough waves in flight to hide the latency of
// the FP64 sequences (rsqrt, sincos, table polynomials) that dominate here.

// Sum over the four lanes of a lane quad (all four active), the same in each lane.
__device__ __forceinline__ double quad_sum(double v) {
  v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  return dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
}

constexpr int kPartSums = 5;   // kinetic, e-e real space, e-I real space, e-e reciprocal, e-I reciprocal


__host__ __device__ inline MeasureLayout measure_layout(int N, int np) {
  MeasureLayout L;
  L.nloc = (N + np - 1) / np;
  // partners split so that the (electron, part) items fill the workgroup about four times
  // over, with at most 512 items: their partial sums are kept in LDS, whose size sets how many
  // workgroups share a compute unit (three at 384 electrons)
  int parts = 1;
  while (parts * L.nloc < 4 * kBlock && parts * 2 * L.nloc <= 512 && parts * 2 <= N) parts *= 2;
  L.parts = parts;
  size_t o = 0;
  L.pos = o; o += sizeof(double) * 3 * N;
  L.ez = o; o += sizeof(double) * 2 * N;
  L.gd = o; o += sizeof(double) * 3 * L.nloc;
  L.ld = o; o += sizeof(double) * L.nloc;
  L.gjp = o; o += sizeof(double) * 3 * (size_t)L.nloc * parts;
  L.ljp = o; o += sizeof(double) * (size_t)L.nloc * parts;
  L.htab = o; o += sizeof(double) * kHTab;
  L.total = o;
  return L;
}

// sum_l B[l][k] (grad phi_l, lap phi_l)(r) for one electron of an FP64 fallback walker: the
// orbitals are evaluated in FP64 from the table, summed against the column as
// sum_stencil weights * (sum_l B[l][k] c_stencil,l), so no FP32-rounded row enters.
// bcol: column k of the FP64 inverse (stride n).
template <typename T>
__device__ void det_terms_fp64(const SysParams& P, const T* __restrict__ table, double x, double y, double z,
                               const double* __restrict__ bcol, int n, double& gx, double& gy, double& gz,
                               double& l2) {
  Axis ax, ay, az;
  axis_weights(x, P.L, P.gx, ax);
  axis_weights(y, P.L, P.gy, ay);
  axis_weights(z, P.L, P.gz, az);
  gx = gy = gz = l2 = 0.0;
  // the weights picked by selects, not by indexing (an indexed private array lives in scratch)
  auto pick = [](const auto (&v)[4], int q) { return q == 0 ? v[0] : (q == 1 ? v[1] : (q == 2 ? v[2] : v[3])); };
#pragma unroll 1
  for (int a = 0; a < 4; ++a) {
    const int ia = pick(ax.idx, a);
    const double wa = pick(ax.w, a), da = pick(ax.dw, a), d2a = pick(ax.d2w, a);
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
      const int ib = pick(ay.idx, b);
      const double wb = pick(ay.w, b), db = pick(ay.dw, b), d2b = pick(ay.d2w, b);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T* cf = table + (((size_t)ia * P.gy + ib) * P.gz + az.idx[c]) * P.S;
        double d = 0.0;
        for (int l = 0; l < n; ++l) d += bcol[(size_t)l * n] * (double)cf[l];
        gx += da * wb * az.w[c] * d;
        gy += wa * db * az.w[c] * d;
        gz += wa * wb * az.dw[c] * d;
        l2 += (d2a * wb * az.w[c] + wa * d2b * az.w[c] + wa * wb * az.d2w[c]) * d;
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void measure_part(const SysParams& P, const Walkers<T>& Wk, const EwaldParams& E,
                                             double* __restrict__ partial, int w, int p, int np) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Jastrow sj;
  __shared__ double red[kPartSums * kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = P.N;
  const MeasureLayout lay = measure_layout(N, np);
  const int nloc = lay.nloc;
  double* spos = reinterpret_cast<double*>(smem + lay.pos);
  double* sez = reinterpret_cast<double*>(smem + lay.ez);
  double* sgd = reinterpret_cast<double*>(smem + lay.gd);
  double* sld = reinterpret_cast<double*>(smem + lay.ld);
  double* sgj = reinterpret_cast<double*>(smem + lay.gjp);
  double* slj = reinterpret_cast<double*>(smem + lay.ljp);
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.jas);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&sj);
    for (int q = tid; q < (int)(sizeof(Jastrow) / 4); q += kBlock) dst[q] = src[q];
  }
  double* shtab = reinterpret_cast<double*>(smem + lay.htab);
  // positions structure-of-arrays: x of every electron, then y, then z
  for (int j = tid; j < 3 * N; j += kBlock) spos[(j % 3) * N + j / 3] = Wk.pos[(size_t)w * 3 * N + j];
  const double* sx = spos;
  const double* sy = spos + N;
  const double* sz = spos + 2 * N;
  if (E.enabled)
    for (int j = tid; j < kHTab; j += kBlock) shtab[(j % (kHDeg + 1)) * kTabInt + j / (kHDeg + 1)] = E.htab[j];
  __syncthreads();
  const double g0 = 2.0 * kPi / P.L, invL = 1.0 / P.L;
  if (E.enabled)
    for (int i = tid; i < N; i += kBlock) {
      double s, c;
      sincos(g0 * sz[i], &s, &c);
      sez[2 * i] = c;
      sez[2 * i + 1] = s;
    }

  // (1) determinant part of this part's electrons i = p nloc + li, one thread per electron:
  // column k of the inverse is read across the threads of consecutive electrons (coalesced),
  // each thread walking its own value/gradient/Laplacian row.  An FP64 fallback walker of the
  // mixed path takes its FP64 inverse and orbitals evaluated in FP64 instead.
  const bool fb64 = Wk.fb && Wk.fb[w];
  for (int li = tid; li < nloc; li += kBlock) {
    const int i = p * nloc + li;
    if (i >= N) break;
    const int sp = i < P.n_up ? 0 : 1;
    const int n = sp ? P.n_dn : P.n_up, k = i - (sp ? P.n_up : 0);
    if (fb64) {
      const double* bcol = Wk.binv64 + (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0) + k;
      double gx, gy, gz, l2;
      det_terms_fp64<T>(P, Wk.table, sx[i], sy[i], sz[i], bcol, n, gx, gy, gz, l2);
      sgd[3 * li] = gx; sgd[3 * li + 1] = gy; sgd[3 * li + 2] = gz; sld[li] = l2;
      continue;
    }
    const size_t item = (size_t)w * N + i;
    const T* row = Wk.vgl + ((size_t)Wk.cur[item] * P.W * N + item) * kComp * P.S;
    const T* B = (Wk.xinv ? Wk.xinv : Wk.binv) + (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0) + k;
    double gx = 0.0, gy = 0.0, gz = 0.0, l2 = 0.0;
    // the row read in 16-byte vectors (S and the rows are 16-byte aligned): every lane reads its
    // own row, so each load instruction touches one line per lane whatever its width
    constexpr int V = 16 / sizeof(T);
    typedef T vec_t __attribute__((ext_vector_type(V)));
    const int nv = n - n % V;
    for (int l0 = 0; l0 < nv; l0 += V) {
      const vec_t rx = *reinterpret_cast<const vec_t*>(row + P.S + l0);
      const vec_t ry = *reinterpret_cast<const vec_t*>(row + 2 * P.S + l0);
      const vec_t rz = *reinterpret_cast<const vec_t*>(row + 3 * P.S + l0);
      const vec_t rl = *reinterpret_cast<const vec_t*>(row + 4 * P.S + l0);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const double b = (double)B[(size_t)(l0 + e) * n];
        gx += b * (double)rx[e];
        gy += b * (double)ry[e];
        gz += b * (double)rz[e];
        l2 += b * (double)rl[e];
      }
    }
    for (int l = nv; l < n; ++l) {
      const double b = (double)B[(size_t)l * n];
      gx += b * (double)row[P.S + l];
      gy += b * (double)row[2 * P.S + l];
      gz += b * (double)row[3 * P.S + l];
      l2 += b * (double)row[4 * P.S + l];
    }
    sgd[3 * li] = gx; sgd[3 * li + 1] = gy; sgd[3 * li + 2] = gz; sld[li] = l2;
  }

  // (2) Jastrow gradient and Laplacian: (electron, part) items, partners j = part (mod parts)
  const int parts = lay.parts;
  for (int q = tid; q < nloc * parts; q += kBlock) {
    const int li = q % nloc, part = q / nloc, i = p * nloc + li;
    if (i >= N) continue;
    const double xi = sx[i], yi = sy[i], zi = sz[i];
    const bool up_i = i < P.n_up;
    double g[3] = {0.0, 0.0, 0.0}, lj = 0.0;
    // partners j = part (mod parts) in three ranges, each with its own radial function:
    // same-spin electrons, opposite-spin electrons, ions
    auto range = [&](const Radial& R, int lo, int hi, auto&& at) {
      for (int j = lo + ((part - lo) % parts + parts) % parts; j < hi; j += parts) {
        double cx, cy, cz;
        at(j, cx, cy, cz);
        const double dx = min_image(xi - cx, P.L, invL), dy = min_image(yi - cy, P.L, invL);
        const double dz = min_image(zi - cz, P.L, invL);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double ri = rsqrt(r2), r = r2 * ri;
        double u, du, d2u;
        radial_eval(R, r, u, du, d2u);
        const double f = j == i ? 0.0 : du * ri;   // no self term
        g[0] += f * dx; g[1] += f * dy; g[2] += f * dz;
        lj += j == i ? 0.0 : d2u + 2.0 * f;
      }
    };
    auto elec = [&](int j, double& cx, double& cy, double& cz) { cx = sx[j]; cy = sy[j]; cz = sz[j]; };
    auto ion = [&](int j, double& cx, double& cy, double& cz) {
      const double* c = P.ions + 4 * (size_t)(j - N);
      cx = c[0]; cy = c[1]; cz = c[2];
    };
    range(up_i ? sj.same : sj.opp, 0, P.n_up, elec);
    range(up_i ? sj.opp : sj.same, P.n_up, N, elec);
    if (P.n_ions > 0) range(sj.ei, N, N + P.n_ions, ion);
    if (P.j3_on) {
      // three-body terms (a = r_iI, c = r_ij at fixed b = r_jI): grad_i u = u_a a^ + u_c c^,
      // lap_i u = u_aa + 2 u_a / a + u_cc + 2 u_c / c + 2 u_ac a^.c^; partners j = part (mod parts)
      const double h = P.j3_h;
      // ions near electron i (a < h), ascending; with at most 64 ions a lane visits only its own
      // near ions instead of every ion some lane of the wave is near
      uint64_t near = 0;
      const bool masked = P.n_ions <= 64;
      if (masked)
        for (int I = 0; I < P.n_ions; ++I) {
          const double* ion = P.ions + 4 * (size_t)I;
          const double ax = min_image(xi - ion[0], P.L, invL), ay = min_image(yi - ion[1], P.L, invL);
          const double az = min_image(zi - ion[2], P.L, invL);
          if (sqrt(ax * ax + ay * ay + az * az) < h) near |= 1ull << I;
        }
      for (int I = masked ? (near ? __builtin_ctzll(near) : P.n_ions) : 0; I < P.n_ions;
           I = masked ? ((near &= near - 1) ? __builtin_ctzll(near) : P.n_ions) : I + 1) {
        const double* ion = P.ions + 4 * (size_t)I;
        const double ax = min_image(xi - ion[0], P.L, invL), ay = min_image(yi - ion[1], P.L, invL);
        const double az = min_image(zi - ion[2], P.L, invL);
        const double a = sqrt(ax * ax + ay * ay + az * az);
        if (a >= h) continue;
        for (int j = part; j < N; j += parts) {
          if (j == i) continue;
          const double bx = min_image(sx[j] - ion[0], P.L, invL), by = min_image(sy[j] - ion[1], P.L, invL);
          const double bz = min_image(sz[j] - ion[2], P.L, invL);
          const double b = sqrt(bx * bx + by * by + bz * bz);
          if (b >= h) continue;
          const double cx = min_image(xi - sx[j], P.L, invL), cy = min_image(yi - sy[j], P.L, invL);
          const double cz = min_image(zi - sz[j], P.L, invL);
          const double c = sqrt(cx * cx + cy * cy + cz * cz);
          double d[6];
          u3_derivs(P, up_i == (j < P.n_up), a, b, c, d);
          const double fa = d[1] / a, fc = d[2] / c;
          g[0] += fa * ax + fc * cx; g[1] += fa * ay + fc * cy; g[2] += fa * az + fc * cz;
          const double ac = (ax * cx + ay * cy + az * cz) / (a * c);
          lj += d[3] + 2.0 * fa + d[4] + 2.0 * fc + 2.0 * d[5] * ac;
        }
      }
    }
    double* gp = sgj + 3 * ((size_t)part * nloc + li);
    gp[0] = g[0]; gp[1] = g[1]; gp[2] = g[2];
    slj[(size_t)part * nloc + li] = lj;
  }

  // (3) Coulomb terms: part p takes the p-th of np contiguous blocks of each pair list, its
  // threads consecutive items (consecutive electrons i, read from consecutive LDS banks)
  double vee = 0.0, vei = 0.0, vee_k = 0.0, vei_k = 0.0;
  if (E.enabled) {
    const double rcut2 = E.rcut * E.rcut;
    // (3a) electron pairs, each once: j = i + d (mod N), d = 1..(N-1)/2, and d = N/2 for i < N/2
    const int D = (N - 1) / 2;
    const int n_pairs = N * D + ((N % 2 == 0) ? N / 2 : 0);
    const int qa0 = (int)((long)n_pairs * p / np), qa1 = (int)((long)n_pairs * (p + 1) / np);
    for (int q = qa0 + tid; q < qa1; q += kBlock) {
      int i, j;
      if (q < N * D) { i = q % N; j = i + q / N + 1; if (j >= N) j -= N; }
      else { i = q - N * D; j = i + N / 2; }
      const double dx = min_image(sx[i] - sx[j], P.L, invL);
      const double dy = min_image(sy[i] - sy[j], P.L, invL);
      const double dz = min_image(sz[i] - sz[j], P.L, invL);
      vee += screened_images(dx, dy, dz, P.L, E.kappa, rcut2, shtab);
    }
    // (3b) electron-ion pairs
    const int n_ei = N * P.n_ions;
    const int qb0 = (int)((long)n_ei * p / np), qb1 = (int)((long)n_ei * (p + 1) / np);
    for (int q = qb0 + tid; q < qb1; q += kBlock) {
      const int i = q % N, I = q / N;
      const double* ion = P.ions + 4 * I;
      const double dx = min_image(sx[i] - ion[0], P.L, invL);
      const double dy = min_image(sy[i] - ion[1], P.L, invL);
      const double dz = min_image(sz[i] - ion[2], P.L, invL);
      vei -= ion[3] * screened_images(dx, dy, dz, P.L, E.kappa, rcut2, shtab);
    }
    // (3c) reciprocal space: items (segment, quarter of the electrons) in lane quads; a
    // segment holds at most kSeg vectors of one (Gx, Gy) column.  Each lane sums e^{iG.r}
    // over its quarter (one sincos per electron, then the Gz recurrence), the quad adds its
    // four partial structure factors, and the quad's first lane adds w(G) |S|^2 and the
    // cross term with the ions.  Quads are active or idle as a whole.
    for (int u = tid; p + np * (u >> 2) < E.n_seg; u += kBlock) {
      const int q = p + np * (u >> 2), c4 = u & 3;
      const int* seg = E.segs + 5 * q;
      const int mx = seg[0], my = seg[1], lo = seg[2], cnt = seg[3] - seg[2] + 1, goff = seg[4];
      double sr[kSeg], si[kSeg];
#pragma unroll
      for (int m = 0; m < kSeg; ++m) { sr[m] = 0.0; si[m] = 0.0; }
      for (int i = c4; i < N; i += 4) {
        double br, bi;
        sincos(g0 * (mx * sx[i] + my * sy[i] + lo * sz[i]), &bi, &br);
        const double er = sez[2 * i], ei = sez[2 * i + 1];
#pragma unroll
        for (int m = 0; m < kSeg; ++m) {
          sr[m] += br;
          si[m] += bi;
          const double t = br * er - bi * ei;
          bi = br * ei + bi * er;
          br = t;
        }
      }
#pragma unroll
      for (int m = 0; m < kSeg; ++m) {
        sr[m] = quad_sum(sr[m]);
        si[m] = quad_sum(si[m]);
      }
      if (c4 == 0) {
#pragma unroll
        for (int m = 0; m < kSeg; ++m) {
          if (m < cnt) {
            const double* gv = E.gvec + 4 * (goff + m);
            const double re = -sr[m], im = -si[m];   // electron charge -1
            vee_k += gv[3] * (re * re + im * im);
            vei_k += gv[3] * 2.0 * (re * E.s_ion[2 * (goff + m)] + im * E.s_ion[2 * (goff + m) + 1]);
          }
        }
      }
    }
  }
  __syncthreads();

  // (4) per-electron kinetic term from (1) and (2)
  double tkin = 0.0;
  for (int li = tid; li < nloc; li += kBlock) {
    if (p * nloc + li >= N) break;
    double g[3] = {0.0, 0.0, 0.0}, lj = 0.0;
    for (int part = 0; part < parts; ++part) {
      const double* gp = sgj + 3 * ((size_t)part * nloc + li);
      g[0] += gp[0]; g[1] += gp[1]; g[2] += gp[2];
      lj += slj[(size_t)part * nloc + li];
    }
    const double dot = sgd[3 * li] * g[0] + sgd[3 * li + 1] * g[1] + sgd[3 * li + 2] * g[2];
    tkin += -0.5 * (sld[li] + 2.0 * dot + lj + g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  }
  const double a = wave_sum_dpp(tkin), b = wave_sum_dpp(vee), c = wave_sum_dpp(vei);
  const double d = wave_sum_dpp(vee_k), e = wave_sum_dpp(vei_k);
  if (lane == 0) {
    red[wave] = a; red[kWaves + wave] = b; red[2 * kWaves + wave] = c;
    red[3 * kWaves + wave] = d; red[4 * kWaves + wave] = e;
  }
  __syncthreads();
  if (tid < kPartSums) {
    double t = 0.0;
    for (int q = 0; q < kWaves; ++q) t += red[tid * kWaves + q];
    partial[((size_t)w * np + p) * kPartSums + tid] = t;
  }
}

// out[w] = (T, V_ee, V_eI, V_II) from the parts' partial sums, added in part order.
__device__ __forceinline__ void measure_finish(const EwaldParams& E, const double* __restrict__ partial,
                                               double* __restrict__ out, int w, int np) {
  double t = 0.0, x = 0.0, y = 0.0, xk = 0.0, yk = 0.0;
  for (int p = 0; p < np; ++p) {
    const double* q = partial + ((size_t)w * np + p) * kPartSums;
    t += q[0]; x += q[1]; y += q[2]; xk += q[3]; yk += q[4];
  }
  out[4 * w + 0] = t;
  out[4 * w + 1] = E.enabled ? (x + xk) + E.c_ee : 0.0;
  out[4 * w + 2] = E.enabled ? (y + yk) + E.c_ei : 0.0;
  out[4 * w + 3] = E.enabled ? E.v_ii : 0.0;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_measure(SysParams P, Walkers<T> Wk, EwaldParams E,
                                                    double* __restrict__ partial, int np) {
  measure_part<T>(P, Wk, E, partial, blockIdx.x / np, blockIdx.x % np, np);
}

__global__ __launch_bounds__(kBlock) void k_measure_finish(EwaldParams E, const double* __restrict__ partial,
                                                           double* __restrict__ out, int W, int np) {
  const int w = blockIdx.x * kBlock + threadIdx.x;
  if (w < W) measure_finish(E, partial, out, w, np);
}

// Batched: block b computes part bmap[b].y % np of walker bmap[b].y / np of system bmap[b].x.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_measure_batched(const SysDev<T>* __restrict__ sd,
                                                            const int2* __restrict__ bmap) {
  __shared__ SysDev<T> s;
  const int2 m = bmap[blockIdx.x];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(sd + m.x);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&s);
    for (int q = threadIdx.x; q < (int)(sizeof(SysDev<T>) / 4); q += kBlock) dst[q] = src[q];
  }
  __syncthreads();
  measure_part<T>(s.P, s.W, s.E, s.mpart, m.y / s.np, m.y % s.np, s.np);
}

// Batched finish: thread t handles (system, walker) fmap[t].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_measure_finish_batched(const SysDev<T>* __restrict__ sd,
                                                                   const int2* __restrict__ fmap, int n) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int2 m = fmap[t];
  const SysDev<T>& s = sd[m.x];
  measure_finish(s.E, s.mpart, s.eout, m.y, s.np);
}

int measure_parts(int W) {
  // aim at about eight workgroups per compute unit over the whole launch
  int np = 1;
  while (np < 8 && (long)W * np < 2048) np *= 2;
  return np;
}

size_t measure_lds_bytes(const SysParams& P, int np) { return measure_layout(P.N, np).total; }

template <typename T>
hipError_t launch_measure_batched(const SysDev<T>* sd, const int2* bmap, int n_blocks, const int2* fmap,
                                  int n_walkers, size_t lds, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (lds > 65536) {
    const hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_measure_batched<T>));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_measure_batched<T>, dim3(n_blocks), dim3(kBlock), lds, st, sd, bmap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_measure_finish_batched<T>, dim3((n_walkers + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                     sd, fmap, n_walkers);
  return hipGetLastError();
}

template hipError_t launch_measure_batched<double>(const SysDev<double>*, const int2*, int, const int2*, int,
                                                   size_t, hipStream_t);
template hipError_t launch_measure_batched<float>(const SysDev<float>*, const int2*, int, const int2*, int,
                                                  size_t, hipStream_t);

template <typename T>
hipError_t launch_measure(const SysParams& P, const Walkers<T>& Wk, const EwaldParams& E, double* partial,
                          double* out, hipStream_t st) {
  const int np = measure_parts(P.W);
  const size_t bytes = measure_layout(P.N, np).total;
  if (bytes > 65536) {
    const hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_measure<T>));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_measure<T>, dim3(P.W * np), dim3(kBlock), bytes, st, P, Wk, E, partial, np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_measure_finish, dim3((P.W + kBlock - 1) / kBlock), dim3(kBlock), 0, st, E, partial, out,
                     P.W, np);
  return hipGetLastError();
}

template hipError_t launch_measure<double>(const SysParams&, const Walkers<double>&, const EwaldParams&, double*,
                                           double*, hipStream_t);
template hipError_t launch_measure<float>(const SysParams&, const Walkers<float>&, const EwaldParams&, double*,
                                          double*, hipStream_t);

hipError_t measure_lds_limits() {
  const void* ks[] = {reinterpret_cast<const void*>(&k_measure<double>), reinterpret_cast<const void*>(&k_measure<float>),
                      reinterpret_cast<const void*>(&k_measure_batched<double>),
                      reinterpret_cast<const void*>(&k_measure_batched<float>)};
  for (const void* k : ks) {
    const hipError_t e = allow_dynamic_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qmc
