/*
 * sanitize_check.c -- TEST INFRASTRUCTURE: a stand-alone driver of the oracle
 * for an AddressSanitizer / UndefinedBehaviorSanitizer build (host code only).
 * tests/test_oracle_sanitized.py compiles it together with m2m_oracle.c under
 * -fsanitize=address,undefined and runs it; any report fails the test.
 *
 * It steps small models through every branch of the oracle's step: the three
 * analytic potentials and the multipole potential, shells, annuli, a sky grid,
 * line-of-sight moments 0..2 and Gauss-Hermite h1..h4, flat and moving
 * histogram priors (both second axes, with and without Lz/L), both update laws,
 * frozen particles, and discrete tracers.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "m2m_oracle.c"

static uint64_t lcg = 12076403u;
static double urand(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) / 9007199254740992.0;
}

static int run_case(int pot_kind, int prior_kind, int ax2, int n2, int update, int frozen, int tracers) {
    const int64_t N = 600;
    or_cfg c;
    memset(&c, 0, sizeof c);
    c.N = N;
    c.dt = 0.01; c.eps = 1e-4; c.mu = 1e-2; c.tau = 0.5;
    c.update = (int16_t)update; c.frozen = (int16_t)frozen;
    c.pot.kind = pot_kind;
    c.pot.G = 1.0; c.pot.M = 1.0; c.pot.a = 1.0;
    c.pot.v0 = 1.0; c.pot.Rc = 0.1; c.pot.q = 0.8;
    c.pot.Mh = 3.0; c.pot.rs = 2.0;
    c.pot.lmax = 4; c.pot.nnode = 40; c.pot.rmin = 1e-2; c.pot.rmax = 50.0; c.pot.Mtot = 1.0;
    static double eshell[11], eann[9], gh[2 * 8];
    for (int k = 0; k <= 10; ++k) eshell[k] = 0.1 * pow(100.0, k / 10.0);
    for (int k = 0; k <= 8; ++k) eann[k] = 0.1 * pow(50.0, k / 8.0);
    for (int k = 0; k < 8; ++k) { gh[k] = 0.02 * k; gh[8 + k] = 0.3 + 0.05 * k; }
    or_layout *L = &c.lay;
    L->incl = 0.7; L->nbin = 4;
    L->kind[0] = OR_BIN_SHELL; L->nmom[0] = 1; L->mom[0][0] = 0; L->nedge[0] = 11; L->edge[0] = eshell;
    L->kind[1] = OR_BIN_ANNULUS; L->nmom[1] = 3; L->mom[1][0] = 0; L->mom[1][1] = 1; L->mom[1][2] = 2;
    L->nedge[1] = 9; L->edge[1] = eann;
    L->kind[2] = OR_BIN_ANNULUS; L->nmom[2] = 3; L->mom[2][0] = 3; L->mom[2][1] = 5; L->mom[2][2] = 6;
    L->nedge[2] = 9; L->edge[2] = eann; L->gh[2] = gh;
    L->kind[3] = OR_BIN_GRID; L->nmom[3] = 2; L->mom[3][0] = 0; L->mom[3][1] = 4; L->gh[3] = NULL;
    L->nx[3] = 6; L->ny[3] = 5; L->x0[3] = -3; L->x1[3] = 3; L->y0[3] = -2.5; L->y1[3] = 2.5;
    static double gh3[2 * 30];
    for (int k = 0; k < 30; ++k) { gh3[k] = 0.0; gh3[30 + k] = 0.5; }
    L->gh[3] = gh3;
    int J = 10 + 3 * 8 + 3 * 8 + 2 * 30;
    c.J = J;
    double *Y = calloc(J, sizeof(double)), *sig = calloc(J, sizeof(double));
    for (int j = 0; j < J; ++j) { Y[j] = 0.01 * (1 + j % 7); sig[j] = 0.01; }
    c.Y = Y; c.sigma = sig;
    c.prior.kind = prior_kind; c.prior.ax2 = ax2;
    c.prior.n[0] = 8; c.prior.n[1] = 6; c.prior.n[2] = n2; c.prior.period = 2;
    c.prior.Emin = pot_kind == OR_POT_LOG ? -1.0 : -1.2; c.prior.Emax = pot_kind == OR_POT_LOG ? 3.0 : -0.01;
    c.prior.flat_value = 1.0 / N;
    c.prior.ref = c.pot;
    if (pot_kind == OR_POT_MULTIPOLE) { c.prior.ref.kind = OR_POT_LOG; c.prior.Emin = -1.0; c.prior.Emax = 3.0; }
    int32_t tb[40];
    double tv[40], ts[40];
    c.trc.binning = -1;
    if (tracers) {
        for (int t = 0; t < 40; ++t) { tb[t] = t % 8; tv[t] = 0.3 * (urand() - 0.5); ts[t] = 0.1; }
        c.trc.binning = 1; c.trc.n = 40; c.trc.bin = tb; c.trc.v = tv; c.trc.s = ts; c.trc.lambda = 0.5;
    }
    or_state s;
    memset(&s, 0, sizeof s);
    double *buf = calloc((size_t)N * 8 + 3 * (size_t)J, sizeof(double));
    s.x = buf; s.y = buf + N; s.z = buf + 2 * N; s.vx = buf + 3 * N; s.vy = buf + 4 * N; s.vz = buf + 5 * N;
    s.w = buf + 6 * N; s.what = buf + 7 * N;
    s.ys = buf + 8 * N; s.yobs = s.ys + J; s.delta = s.yobs + J;
    int nlm = (c.pot.lmax + 1) * (c.pot.lmax + 1);
    s.mpA = calloc((size_t)c.pot.nnode * nlm, sizeof(double));
    s.mpB = calloc((size_t)c.pot.nnode * nlm, sizeof(double));
    s.tL = calloc(40, sizeof(double)); s.tLobs = calloc(40, sizeof(double));
    s.tM = calloc(8, sizeof(double)); s.tMobs = calloc(8, sizeof(double));
    for (int64_t i = 0; i < N; ++i) {
        double r = 0.05 + 4.0 * urand(), ct = 2 * urand() - 1, ph = 6.283185307179586 * urand();
        double st = sqrt(1 - ct * ct);
        s.x[i] = r * st * cos(ph); s.y[i] = r * st * sin(ph); s.z[i] = r * ct;
        s.vx[i] = 0.3 * (urand() - 0.5); s.vy[i] = 0.3 * (urand() - 0.5); s.vz[i] = 0.3 * (urand() - 0.5);
        s.w[i] = 1.0 / N;
        s.what[i] = 1.0 / N;
    }
    if (pot_kind == OR_POT_MULTIPOLE) or_mp_coeffs(&c.pot, N, s.x, s.y, s.z, s.w, s.mpA, s.mpB);
    double stats[8 * 6];
    int rc = or_run(&c, &s, 6, stats);
    for (int k = 0; k < 6 * 8; ++k)
        if (!isfinite(stats[k])) rc = 99;
    free(Y); free(sig); free(buf); free(s.mpA); free(s.mpB);
    free(s.tL); free(s.tLobs); free(s.tM); free(s.tMobs);
    return rc;
}

int main(void) {
    int bad = 0, cases = 0;
    for (int pot = 0; pot <= 3; ++pot)
        for (int pk = 0; pk <= 1; ++pk)
            for (int ax2 = 0; ax2 <= 1; ++ax2)
                for (int n2 = 1; n2 <= 4; n2 += 3)
                    for (int upd = 0; upd <= 1; ++upd) {
                        int rc = run_case(pot, pk, ax2, n2, upd, (pot + upd) % 3 == 0, (pk + ax2 + upd) % 2);
                        ++cases;
                        if (rc != 0 && rc != OR_NONPOSITIVE) {
                            printf("case pot %d prior %d ax2 %d n2 %d update %d: rc %d\n", pot, pk, ax2, n2, upd, rc);
                            bad = 1;
                        }
                    }
    printf("%d cases %s\n", cases, bad ? "FAILED" : "ok");
    return bad;
}
