/*
 * Host-side memory and undefined-behaviour check of the oracle: compiled together with
 * oracle/qmc_oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitized.py, it runs every move kind, the measurement and DMC on two
 * small systems (a plane-wave electron gas and a spline solid with ions, one-, two- and
 * three-body Jastrow factors) and exits 0 when every call succeeded.
 */
#include <stdio.h>

#include "../../oracle/qmc_oracle.c"

static uint64_t lcg_state = 12345u;
static double lcg_uniform(void) {
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * 0x1.0p-53;
}

static int run_all(orc_system* s, const char* name) {
    const int N = s->n_up + s->n_dn, W = 3, S = 3;
    int32_t ids[3] = {0, 1, 2};
    double* energies = (double*)calloc((size_t)W * S * 4, sizeof(double));
    uint8_t* bits = (uint8_t*)calloc((size_t)W * S * N, 1);
    double* trace = (double*)calloc((size_t)W * S * N * 3, sizeof(double));
    double* fpos = (double*)calloc((size_t)W * N * 3, sizeof(double));
    double ld[6], ldlu[6];
    int32_t sg[6];
    for (int kind = 0; kind < 4; ++kind) {
        s->all_electron = kind;
        const int rc = orc_vmc_run(s, W, ids, NULL, 0, S, 1, energies, bits, trace, fpos, ld, sg, ldlu, 2);
        if (rc) { printf("%s: vmc kind %d returned %d\n", name, kind, rc); return 1; }
        for (int q = 0; q < W * S * 4; ++q)
            if (!isfinite(energies[q])) { printf("%s: non-finite energy (kind %d)\n", name, kind); return 1; }
    }
    for (int kind = 2; kind < 4; ++kind) {
        s->all_electron = kind;
        const int slots = 8, target = 6, steps = 3;
        double* st = (double*)calloc((size_t)steps * 6, sizeof(double));
        double* w = (double*)calloc((size_t)steps * slots, sizeof(double));
        double* en = (double*)calloc((size_t)steps * slots, sizeof(double));
        int32_t* m = (int32_t*)calloc((size_t)steps * slots, sizeof(int32_t));
        int32_t* pl = (int32_t*)calloc((size_t)steps * slots, sizeof(int32_t));
        double* fp = (double*)calloc((size_t)slots * N * 3, sizeof(double));
        int32_t* fs = (int32_t*)calloc((size_t)slots, sizeof(int32_t));
        const int rc = orc_dmc_run(s, slots, target, NAN, 0.5, 0, steps, st, w, m, pl, en, fp, fs, 2);
        free(st); free(w); free(en); free(m); free(pl); free(fp); free(fs);
        if (rc) { printf("%s: dmc kind %d returned %d\n", name, kind, rc); return 1; }
    }
    free(energies); free(bits); free(trace); free(fpos);
    return 0;
}

int main(void) {
    /* 14-electron gas: the closed shell |n|^2 <= 1 of real plane waves, Pade two-body Jastrow */
    {
        orc_system s;
        memset(&s, 0, sizeof s);
        s.n_up = s.n_dn = 7;
        s.L = 3.88513;
        s.spo_kind = ORC_SPO_PLANEWAVE;
        s.n_orb = 7;
        double k[21] = {0};
        int32_t kind[7] = {0, 0, 1, 0, 1, 0, 1};
        for (int a = 0; a < 3; ++a) {
            k[3 * (1 + 2 * a) + a] = 2.0 * ORC_PI / s.L;
            k[3 * (2 + 2 * a) + a] = 2.0 * ORC_PI / s.L;
        }
        s.pw_k = k;
        s.pw_kind = kind;
        s.j2_kind = ORC_J_PADE;
        s.j2_a = 0.5;
        s.j2_b = 1.0;
        s.sigma = 0.3;
        s.seed = 7;
        s.coulomb = 1;
        if (run_all(&s, "electron gas")) return 1;
    }
    /* spline solid: 10 electrons (5 + 5), 8^3 table, two ions, B-spline J1 and J2, three-body term */
    {
        orc_system s;
        memset(&s, 0, sizeof s);
        s.n_up = 5; s.n_dn = 5;
        s.L = 4.2;
        s.spo_kind = ORC_SPO_SPLINE;
        s.n_orb = 5;
        s.gx = s.gy = s.gz = 8;
        double* coefs = (double*)malloc(sizeof(double) * 8 * 8 * 8 * 5);
        for (int q = 0; q < 8 * 8 * 8 * 5; ++q) coefs[q] = 2.0 * lcg_uniform() - 1.0;
        s.coefs = coefs;
        double ions[6] = {1.0, 1.2, 0.8, 3.0, 2.9, 3.1}, Z[2] = {3.0, 2.0};
        s.n_ions = 2; s.ion_pos = ions; s.ion_Z = Z;
        double p2[8], p1[8];
        for (int q = 0; q < 8; ++q) { p2[q] = -0.4 * pow(1.0 - q / 7.0, 3); p1[q] = -0.3 * pow(1.0 - q / 7.0, 3); }
        s.j2_kind = ORC_J_BSPLINE; s.j2_M = 8; s.j2_rc = s.L / 2; s.j2_p = p2;
        s.j2_cusp_same = 0.25; s.j2_cusp_opp = 0.5;
        s.j1_kind = ORC_J_BSPLINE; s.j1_M = 8; s.j1_rc = s.L / 2; s.j1_p = p1; s.j1_cusp = 0.0;
        double gamma[2 * 3 * 3 * 3];
        for (int q = 0; q < 54; ++q) gamma[q] = 0.01 * (2.0 * lcg_uniform() - 1.0);
        s.j3_mei = 2; s.j3_mee = 2; s.j3_rc = s.L / 2; s.j3_gamma = gamma;
        s.sigma = 0.25;
        s.seed = 11;
        s.coulomb = 1;
        const int rc = run_all(&s, "spline solid");
        free(coefs);
        if (rc) return 1;
    }
    printf("ok\n");
    return 0;
}
