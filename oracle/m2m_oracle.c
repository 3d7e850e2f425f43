/*
 * m2m_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, FP64 CPU reference of the per-timestep loop of the NMAGIC
 * made-to-measure particle method (Morganti & Gerhard, "NMAGIC made-to-measure
 * particle models of galaxies").  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or table
 * with the GPU library.
 *
 * What the paper fixes:
 *   - merit F = -chi^2/2 + mu S, maximised over the particle weights (section 2, eq. 1);
 *   - pseudo-entropy S = -sum_i w_i ln(w_i / what_i) (section 2, eq. 2);
 *   - the weights are adapted while the particles move in a fixed or
 *     self-consistent potential (section 2);
 *   - flat priors what_i = 1/N and initial weights 1/N (section 2.1);
 *   - moving priors follow the weight distribution over integrals of motion or
 *     approximately conserved quantities (section 2.1).
 * Everything else (integrator, observable kernels, smoothing, update law, prior
 * cells, multipole scheme) is a stated reading of the method; each function
 * below names the reading it implements.
 *
 * One step n, in this order (state: z(t_n), w(n), smoothed y(n-1), what(n-1)):
 *   1 observe   y_j(n)   = sum_i w_i K_j(z_i)
 *   2 smooth    ys_j(n)  = ys_j(n-1) + (dt/tau)(y_j(n) - ys_j(n-1)), ys(-1) = y(0)
 *   3 deviate   D_j(n)   = (ys_j(n) - Y_j)/sigma_j,  chi2 = sum_j D_j^2
 *   4 prior     if n mod P == 0: what_i = mean weight of the particles in i's cell
 *   5 entropy   S(n) = -sum_i w_i ln(w_i/what_i),  F = -chi2/2 + mu S
 *   6 update    G_i = -sum_j K_j(z_i) D_j/sigma_j - mu (ln(w_i/what_i) + 1)
 *               (dw_i/dt = eps w_i dF/dw_i with the priors held fixed), integrated over
 *               dt as w_i <- w_i exp(eps dt G_i) (default) or w_i (1 + eps dt G_i)
 *   7 push      kick-drift-kick leapfrog over dt
 * With discrete tracer velocities (section 1 lists PNe velocities among the
 * data; reading: the likelihood term of NMAGIC's discrete-velocity fits), steps
 * 1-3 also observe, smooth (as y) and score the tracers:
 *   L_t(n) = sum_i w_i [b(z_i) = b_t] phi(v_los,i; V_t, s_t),  M_b(n) = sum_i w_i [b(z_i) = b]
 *   loglike = sum_t ln(Ls_t / Ms_(b_t))  (each tracer's model LOSVD density at V_t)
 * and the update gains lambda d(loglike)/dw_i with the smoothed values held:
 *   G_i += lambda (sum_{t in b(z_i)} phi(v_los,i; V_t, s_t) / Ls_t - n_(b(z_i)) / Ms_(b(z_i)))
 * (phi the normal density, s_t^2 = error^2 + smoothing^2, n_b the tracers in bin b).
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXBIN 4
#define OR_MAXL 16

enum { OR_POT_HERNQUIST = 0, OR_POT_LOG = 1, OR_POT_HNFW = 2, OR_POT_MULTIPOLE = 3 };
enum { OR_BIN_SHELL = 1, OR_BIN_ANNULUS = 2, OR_BIN_GRID = 3 };
enum { OR_PRIOR_FLAT = 0, OR_PRIOR_HIST = 1, OR_PRIOR_EXTERNAL = 2 };
enum { OR_OK = 0, OR_NONPOSITIVE = 4, OR_NONFINITE = 5 };

typedef struct {
    int32_t kind;
    int32_t lmax, nnode, pad;
    double G, M, a, v0, Rc, q, Mh, rs;
    double rmin, rmax, Mtot;
} or_pot;

typedef struct {
    double incl;
    int32_t nbin, pad;
    int32_t kind[OR_MAXBIN];
    int32_t nmom[OR_MAXBIN];
    int32_t mom[OR_MAXBIN][3];
    int32_t nedge[OR_MAXBIN];
    const double *edge[OR_MAXBIN];
    int32_t nx[OR_MAXBIN], ny[OR_MAXBIN];
    double x0[OR_MAXBIN], x1[OR_MAXBIN], y0[OR_MAXBIN], y1[OR_MAXBIN];
    const double *gh[OR_MAXBIN];   /* Gauss-Hermite moments: V_b[nb] then sigma_b[nb] */
} or_layout;

typedef struct {
    int32_t kind;      /* OR_PRIOR_*                                   */
    int32_t ax2;       /* 0: L/Lc(E) in [0,1]; 1: Lz/Lc(E) in [-1,1]   */
    int32_t n[3];      /* cells along E, second axis, Lz/L (1 = unused) */
    int32_t period;
    double Emin, Emax;
    double flat_value;
    or_pot ref;        /* potential in which E and Lc(E) are measured  */
} or_prior;

/* Discrete tracers: per tracer its bin in layout binning `binning`, its
 * line-of-sight velocity and kernel width s_t (sqrt(error^2 + h^2)). */
typedef struct {
    int32_t binning;   /* -1: no tracers */
    int32_t n;
    const int32_t *bin;
    const double *v, *s;
    double lambda;
} or_tracers;

typedef struct {
    int64_t N;
    int32_t J;
    int16_t update;    /* 0: w (1 + eps dt G) (explicit Euler); 1: w exp(eps dt G) */
    int16_t frozen;    /* 1: particles do not move (step 7 skipped)               */
    double dt, eps, mu, tau;
    or_pot pot;
    or_layout lay;
    or_prior prior;
    const double *Y, *sigma;
    or_tracers trc;
} or_cfg;

typedef struct {
    double *x, *y, *z, *vx, *vy, *vz, *w;
    double *what;          /* N: prior per particle                       */
    double *ys;            /* J: smoothed observables                     */
    double *yobs;          /* J: observables of the last observe          */
    double *delta;         /* J: smoothed deviations                      */
    double *mpA, *mpB;     /* multipole coefficient tables (nnode x nlm)  */
    int64_t n;             /* step index                                  */
    double chi2, chi2_inst, S, F, sumw, minw, sumw2;
    int32_t status, pad;
    int64_t bad_step;
    double *tL, *tM;       /* tracers: smoothed L_t (n) and bin masses M_b (nb)  */
    double *tLobs, *tMobs; /* the same from the last observe                     */
    double loglike;
} or_state;

static int nthreads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int or_threads(void) { return nthreads(); }

/* Threads of the parallel loops from now on (the CPU-baseline timing runs the
 * oracle on one core as well as on all of them). */
void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ potentials
 * Section 2: the potential is fixed and known a priori, or self-consistent.
 * Analytic forms: Hernquist Phi = -GM/(r+a); logarithmic
 * Phi = v0^2/2 ln(Rc^2 + R^2 + z^2/q^2); Hernquist + NFW with
 * Phi_NFW = -G Mh ln(1 + r/rs)/r.  The acceleration is zero at r = 0 exactly. */
void or_potential(const or_pot *p, double x, double y, double z,
                  double *phi, double *ax, double *ay, double *az) {
    double r2 = x * x + y * y + z * z, r = sqrt(r2);
    if (p->kind == OR_POT_LOG) {
        double q2 = p->q * p->q;
        double s = p->Rc * p->Rc + x * x + y * y + z * z / q2;
        double v2 = p->v0 * p->v0;
        *phi = 0.5 * v2 * log(s);
        *ax = -v2 * x / s;
        *ay = -v2 * y / s;
        *az = -v2 * z / (q2 * s);
        return;
    }
    /* Hernquist part: dPhi/dr = GM/(r+a)^2 */
    double u = r + p->a;
    double ph = -p->G * p->M / u;
    double dphidr = p->G * p->M / (u * u);
    if (p->kind == OR_POT_HNFW && p->Mh > 0.0) {
        double xx = r / p->rs;
        if (r > 0.0) {
            double l1 = log1p(xx);
            ph += -p->G * p->Mh * l1 / r;
            /* d/dr[-G Mh ln(1+r/rs)/r] = G Mh [ln(1+x)/r^2 - 1/(r (r+rs))] */
            dphidr += p->G * p->Mh * (l1 / r2 - 1.0 / (r * (r + p->rs)));
        } else {
            ph += -p->G * p->Mh / p->rs;
        }
    }
    *phi = ph;
    if (r > 0.0) {
        double f = -dphidr / r;
        *ax = f * x; *ay = f * y; *az = f * z;
    } else {
        *ax = *ay = *az = 0.0;
    }
}

/* Energy of a circular orbit of radius R in the equatorial plane,
 * E_c(R) = Phi(R) + R dPhi/dR / 2, and its angular momentum R v_c. */
static void circular(const or_pot *p, double R, double *Ec, double *Lc) {
    double phi, ax, ay, az;
    or_potential(p, R, 0.0, 0.0, &phi, &ax, &ay, &az);
    double vc2 = -ax * R;           /* R dPhi/dR */
    if (vc2 < 0.0) vc2 = 0.0;
    *Ec = phi + 0.5 * vc2;
    *Lc = R * sqrt(vc2);
}

/* Lc(E): angular momentum of the circular orbit of energy E, by bisection in
 * ln R on [1e-8, 1e8] (E_c(R) increases with R for these potentials).
 * Energies outside the bracket take the end value. */
double or_circular_L(const or_pot *p, double E) {
    double lo = log(1e-8), hi = log(1e8), Ec, Lc;
    circular(p, exp(lo), &Ec, &Lc);
    if (E <= Ec) return Lc;
    circular(p, exp(hi), &Ec, &Lc);
    if (E >= Ec) return Lc;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        circular(p, exp(mid), &Ec, &Lc);
        if (Ec < E) lo = mid; else hi = mid;
        if (hi - lo < 1e-15) break;
    }
    circular(p, exp(0.5 * (lo + hi)), &Ec, &Lc);
    return Lc;
}

/* -------------------------------------------------------------- observables
 * Section 2: chi^2 measures deviations between target and model observables;
 * section 1 lists photometry and line-of-sight kinematics.  Reading: the
 * observables are linear in the weights, y_j = sum_i w_i K_j(z_i), with
 *   shell   K = 1[e_k <= r < e_k+1]               (3D density)
 *   annulus K = 1[e_k <= R < e_k+1] * v_los^m      (projected radius R)
 *   grid    K = 1[(X, Y) in pixel k] * v_los^m     (sky plane)
 * (m = 0, 1, 2; the Gauss-Hermite kernels of gh_kernel replace v_los^m for
 * moment codes 3..6)
 * Sky coordinates for inclination i: X = x, Y = y cos i - z sin i,
 * v_los = vy sin i + vz cos i.  Bins are half-open; a particle outside every bin
 * contributes nothing.  Returns the number of non-zero entries. */
static int edge_bin(const double *e, int ne, double r) {
    if (!(r >= e[0]) || !(r < e[ne - 1])) return -1;
    int k = 0;
    while (k + 1 < ne - 1 && r >= e[k + 1]) ++k;
    return k;
}

/* Bin of the position (x, y, z) in binning b, -1 outside (section 2: each
 * observable is the weighted count, or LOS moment, of the particles in one bin
 * of a binning of the projected or spatial coordinates).  Shells bin the
 * radius r, annuli the projected radius, grids the sky plane (x, y cos i -
 * z sin i) into nx * ny pixels numbered iy * nx + ix. */
static int bin_of(const or_layout *L, int b, double ci, double si, double x, double y, double z) {
    double X = x, Ys = y * ci - z * si;
    if (L->kind[b] == OR_BIN_SHELL)
        return edge_bin(L->edge[b], L->nedge[b], sqrt(x * x + y * y + z * z));
    if (L->kind[b] == OR_BIN_ANNULUS)
        return edge_bin(L->edge[b], L->nedge[b], sqrt(X * X + Ys * Ys));
    double fx = floor((X - L->x0[b]) / (L->x1[b] - L->x0[b]) * L->nx[b]);
    double fy = floor((Ys - L->y0[b]) / (L->y1[b] - L->y0[b]) * L->ny[b]);
    if (fx >= 0 && fx < L->nx[b] && fy >= 0 && fy < L->ny[b])
        return (int)fy * L->nx[b] + (int)fx;
    return -1;
}

/* Gauss-Hermite line-of-sight kinematics (section 1: absorption-line
 * kinematics from long-slit and integral-field spectra).  Reading: the LOSVD of
 * bin b is expanded about the Gaussian of mean V_b and dispersion sigma_b given
 * with the data (van der Marel & Franx 1993); moment code 2 + m (m = 1..4) is the
 * kernel K = 2 sqrt(pi) alpha(nu) H_m(nu), nu = (v_los - V_b)/sigma_b,
 * alpha(nu) = exp(-nu^2/2)/sqrt(2 pi), whose mass-weighted expectation under a
 * Gauss-Hermite LOSVD is h_m.  H_m = Hp_m / sqrt(2^m m!) with the physicists'
 * Hermite polynomials Hp_0 = 1, Hp_1 = 2 nu, Hp_(m+1) = 2 nu Hp_m - 2 m Hp_(m-1). */
static double gh_kernel(int m, double nu) {
    double hm1 = 1.0, h = 2.0 * nu, norm = 2.0;   /* Hp_0, Hp_1, 2^1 1! */
    if (m == 0) { h = 1.0; norm = 1.0; }
    for (int k = 1; k < m; ++k) {
        double hn = 2.0 * nu * h - 2.0 * k * hm1;
        hm1 = h;
        h = hn;
        norm *= 2.0 * (k + 1);
    }
    return 2.0 * sqrt(M_PI) * exp(-0.5 * nu * nu) / sqrt(2.0 * M_PI) * h / sqrt(norm);
}

/* Kernel value of moment code mo of a particle in bin k of binning b:
 * 0 mass, 1 v_los, 2 v_los^2, 3..6 Gauss-Hermite h1..h4. */
static double moment_kernel(const or_layout *L, int b, int k, int mo, double vl) {
    if (mo == 0) return 1.0;
    if (mo == 1) return vl;
    if (mo == 2) return vl * vl;
    int nb = L->kind[b] == OR_BIN_GRID ? L->nx[b] * L->ny[b] : L->nedge[b] - 1;
    double nu = (vl - L->gh[b][k]) / L->gh[b][nb + k];
    return gh_kernel(mo - 2, nu);
}

int or_kernel(const or_layout *L, double x, double y, double z,
              double vx, double vy, double vz, int32_t *jidx, double *Kval) {
    (void)vx;
    double ci = cos(L->incl), si = sin(L->incl);
    double vl = vy * si + vz * ci;
    int cnt = 0, off = 0;
    for (int b = 0; b < L->nbin; ++b) {
        int nb = L->kind[b] == OR_BIN_GRID ? L->nx[b] * L->ny[b] : L->nedge[b] - 1;
        int k = bin_of(L, b, ci, si, x, y, z);
        for (int m = 0; m < L->nmom[b]; ++m) {
            if (k >= 0) {
                jidx[cnt] = off + m * nb + k;
                Kval[cnt] = moment_kernel(L, b, k, L->mom[b][m], vl);
                ++cnt;
            }
        }
        off += L->nmom[b] * nb;
    }
    return cnt;
}

/* Bin of every particle in every binning: bin[b * N + i], -1 outside. */
void or_bins(const or_layout *L, int64_t N, const double *x, const double *y, const double *z, int32_t *bin) {
    double ci = cos(L->incl), si = sin(L->incl);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int b = 0; b < L->nbin; ++b)
            bin[(int64_t)b * N + i] = bin_of(L, b, ci, si, x[i], y[i], z[i]);
}

/* ------------------------------------------------------------------- priors
 * Section 2.1: moving priors follow the phase-space structure of the weight
 * distribution, computed over integrals of motion.  Reading: cells on a grid of
 * E (uniform in [Emin, Emax], clamped to the edge cells), then L/Lc(E) in [0,1]
 * or Lz/Lc(E) in [-1,1], then optionally Lz/L in [-1,1]; every axis is clamped. */
static int clampi(double f, int n) {
    if (!(f >= 0.0)) return 0;           /* also NaN */
    if (f >= n) return n - 1;
    return (int)f;
}

int or_cell(const or_prior *P, double x, double y, double z,
            double vx, double vy, double vz) {
    double phi, ax, ay, az;
    or_potential(&P->ref, x, y, z, &phi, &ax, &ay, &az);
    double E = 0.5 * (vx * vx + vy * vy + vz * vz) + phi;
    double Lx = y * vz - z * vy, Ly = z * vx - x * vz, Lz = x * vy - y * vx;
    double L = sqrt(Lx * Lx + Ly * Ly + Lz * Lz);
    double Lc = or_circular_L(&P->ref, E);
    int iE = clampi((E - P->Emin) / (P->Emax - P->Emin) * P->n[0], P->n[0]);
    int i2;
    if (P->ax2 == 0) i2 = clampi((Lc > 0 ? L / Lc : 0.0) * P->n[1], P->n[1]);
    else i2 = clampi(((Lc > 0 ? Lz / Lc : 0.0) + 1.0) * 0.5 * P->n[1], P->n[1]);
    int i3 = 0;
    if (P->n[2] > 1) i3 = clampi(((L > 0 ? Lz / L : 0.0) + 1.0) * 0.5 * P->n[2], P->n[2]);
    return (iE * P->n[1] + i2) * P->n[2] + i3;
}

int64_t or_ncell(const or_prior *P) { return (int64_t)P->n[0] * P->n[1] * P->n[2]; }

/* The integrals of motion the priors are computed over (section 2.1): E, |L|,
 * Lz and Lc(E), in the prior's reference potential, for every particle. */
void or_integrals(const or_prior *P, int64_t N, const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz,
                  double *E, double *L, double *Lz, double *Lc) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double phi, ax, ay, az;
        or_potential(&P->ref, x[i], y[i], z[i], &phi, &ax, &ay, &az);
        E[i] = 0.5 * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]) + phi;
        double Lx = y[i] * vz[i] - z[i] * vy[i], Ly = z[i] * vx[i] - x[i] * vz[i];
        Lz[i] = x[i] * vy[i] - y[i] * vx[i];
        L[i] = sqrt(Lx * Lx + Ly * Ly + Lz[i] * Lz[i]);
        Lc[i] = or_circular_L(&P->ref, E[i]);
    }
}

/* Cell index of every particle. */
void or_cells(const or_prior *P, int64_t N, const double *x, const double *y, const double *z,
              const double *vx, const double *vy, const double *vz, int32_t *cell) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        cell[i] = or_cell(P, x[i], y[i], z[i], vx[i], vy[i], vz[i]);
}

/* Moving prior (section 2.1, reading): what_i = mean of w_k over the particles k
 * that share particle i's cell.  Also returns the cell sums and counts. */
void or_prior_means(const or_prior *P, int64_t N, const double *x, const double *y,
                    const double *z, const double *vx, const double *vy, const double *vz,
                    const double *w, double *what, double *cell_sum, double *cell_cnt) {
    int64_t nc = or_ncell(P);
    int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    or_cells(P, N, x, y, z, vx, vy, vz, cell);
    for (int64_t c = 0; c < nc; ++c) { cell_sum[c] = 0.0; cell_cnt[c] = 0.0; }
    for (int64_t i = 0; i < N; ++i) { cell_sum[cell[i]] += w[i]; cell_cnt[cell[i]] += 1.0; }
    for (int64_t i = 0; i < N; ++i) what[i] = cell_sum[cell[i]] / cell_cnt[cell[i]];
    free(cell);
}

/* ---------------------------------------------------------------- multipole
 * Section 1/2: the potential can be computed self-consistently from the
 * particles.  Reading: a multipole expansion to l <= lmax built from the
 * addition theorem
 *   1/|x - x'| = sum_l r<^l / r>^(l+1) P_l(cos gamma),
 *   P_l(cos gamma) = sum_m (2 - d_m0) (l-m)!/(l+m)! P_l^m(ct) P_l^m(ct') cos m(ph - ph'),
 * so Phi(x) = -G sum_lm c_lm P_l^m(ct) [cos(m ph) (Ac r^-(l+1) + Bc r^l)
 *                                    + sin(m ph) (As r^-(l+1) + Bs r^l)]
 * with Ac_lm(r) = sum_{r_k < r} m_k r_k^l P_l^m(ct_k) cos(m ph_k) and
 *      Bc_lm(r) = sum_{r_k >= r} m_k r_k^-(l+1) P_l^m(ct_k) cos(m ph_k) (sin for As, Bs).
 * Coefficients are kept at nnode log-spaced node radii in [rmin, rmax], built by
 * per-interval sums plus prefix (A) and suffix (B) scans, and interpolated
 * linearly in ln r.  Radii outside [rmin, rmax] are clamped: the expansion is
 * evaluated at the point moved radially onto the clamped radius.
 * Coefficient index: lm(l, m>=0, cos) = l*l + 2m (m>0: cos at l*l+2m-1, sin at l*l+2m). */
static int lm_index(int l, int m, int s) { return m == 0 ? l * l : l * l + 2 * m - 1 + s; }

/* Associated Legendre P_l^m(x) with the Condon-Shortley phase, standard
 * upward recurrence in l for each m.  P[l*(lmax+1)+m]. */
static void legendre(int lmax, double x, double *P) {
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) pmm *= -(2.0 * m - 1.0) * s;
        P[m * (lmax + 1) + m] = pmm;
        if (m + 1 <= lmax) P[(m + 1) * (lmax + 1) + m] = x * (2.0 * m + 1.0) * pmm;
        for (int l = m + 2; l <= lmax; ++l)
            P[l * (lmax + 1) + m] = ((2.0 * l - 1.0) * x * P[(l - 1) * (lmax + 1) + m]
                                     - (l + m - 1.0) * P[(l - 2) * (lmax + 1) + m]) / (l - m);
    }
}

void or_legendre(int lmax, double x, double *P) { legendre(lmax, x, P); }

static double factorial(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* angular parts of one particle: Yc_lm = P_l^m(ct) cos(m ph), Ys_lm = P_l^m(ct) sin(m ph) */
static void angular(int lmax, double x, double y, double z, double *Y) {
    double r = sqrt(x * x + y * y + z * z);
    double ct = r > 0 ? z / r : 1.0;
    double ph = atan2(y, x);
    double P[(OR_MAXL + 1) * (OR_MAXL + 1)];
    legendre(lmax, ct, P);
    for (int l = 0; l <= lmax; ++l)
        for (int m = 0; m <= l; ++m) {
            double p = P[l * (lmax + 1) + m];
            if (m == 0) Y[lm_index(l, 0, 0)] = p;
            else {
                Y[lm_index(l, m, 0)] = p * cos(m * ph);
                Y[lm_index(l, m, 1)] = p * sin(m * ph);
            }
        }
}

/* A, B at the nodes: A[k*nlm + lm], B[k*nlm + lm], masses m_k = w_k Mtot. */
void or_mp_coeffs(const or_pot *p, int64_t N, const double *x, const double *y, const double *z,
                  const double *w, double *A, double *B) {
    int lmax = p->lmax, nn = p->nnode, nlm = (lmax + 1) * (lmax + 1);
    double lr0 = log(p->rmin), dl = (log(p->rmax) - lr0) / (nn - 1);
    /* interval k in -1..nn-1 stored at k+1; interval k = [r_k, r_k+1) */
    int T = nthreads();
    double *SA = (double *)calloc((size_t)T * (nn + 1) * nlm, sizeof(double));
    double *SB = (double *)calloc((size_t)T * (nn + 1) * nlm, sizeof(double));
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double Y[(OR_MAXL + 1) * (OR_MAXL + 1)];
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            double r = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
            int k;
            if (r < p->rmin) k = -1;
            else {
                k = (int)floor((log(r) - lr0) / dl);
                if (k > nn - 1) k = nn - 1;
                /* node radii exp(lr0 + k dl): move k so that r_k <= r < r_k+1 */
                while (k >= 0 && r < exp(lr0 + k * dl)) --k;
                while (k + 1 <= nn - 1 && r >= exp(lr0 + (k + 1) * dl)) ++k;
            }
            angular(lmax, x[i], y[i], z[i], Y);
            double m = w[i] * p->Mtot;
            double *sa = SA + ((size_t)t * (nn + 1) + (k + 1)) * nlm;
            double *sb = SB + ((size_t)t * (nn + 1) + (k + 1)) * nlm;
            double rl = 1.0;
            for (int l = 0; l <= lmax; ++l) {
                double ra = m * rl, rb = r > 0 ? m / (rl * r) : 0.0;
                for (int j = l * l; j < (l + 1) * (l + 1); ++j) { sa[j] += ra * Y[j]; sb[j] += rb * Y[j]; }
                rl *= r;
            }
        }
    }
    for (int t = 1; t < T; ++t)
        for (size_t e = 0; e < (size_t)(nn + 1) * nlm; ++e) {
            SA[e] += SA[(size_t)t * (nn + 1) * nlm + e];
            SB[e] += SB[(size_t)t * (nn + 1) * nlm + e];
        }
    /* A(r_k) = sum of intervals -1..k-1 ; B(r_k) = sum of intervals k..nn-1 */
    for (int j = 0; j < nlm; ++j) {
        double acc = 0.0;
        for (int k = 0; k < nn; ++k) { acc += SA[(size_t)k * nlm + j]; A[(size_t)k * nlm + j] = acc; }
        acc = 0.0;
        for (int k = nn - 1; k >= 0; --k) { acc += SB[(size_t)(k + 1) * nlm + j]; B[(size_t)k * nlm + j] = acc; }
    }
    free(SA); free(SB);
}

/* Phi and acceleration from coefficient values Ar, Br (already at radius r),
 * with A and B held fixed (the dA/dr and dB/dr terms cancel in the exact
 * expansion).  Written with the solid harmonics R_lm = r^l P_l^m(ct) e^(i m ph),
 *   Phi = -G sum_lm c_lm [Re R_lm (Ac r^-(2l+1) + Bc) + Im R_lm (As r^-(2l+1) + Bs)],
 * so that the gradient has no coordinate singularity on the polar axis:
 *   d/dz R_lm = (l+m) R_(l-1)m,  (d/dx + i d/dy) R_lm = R_(l-1)(m+1),
 *   (d/dx - i d/dy) R_lm = -(l+m)(l+m-1) R_(l-1)(m-1)  (m >= 1; for m = 0 it is the
 *   complex conjugate of (d/dx + i d/dy) R_l0, R_l0 being real),
 * identities of the associated Legendre functions with the Condon-Shortley phase.
 * R_lm follows from P_m^m = (-1)^m (2m-1)!! st^m and the recurrence in l. */
static void mp_field(int lmax, double G, double x, double y, double z,
                     const double *Ar, const double *Br,
                     double *phi, double *ax, double *ay, double *az) {
    const int L1 = OR_MAXL + 1;
    double Rre[(OR_MAXL + 1) * (OR_MAXL + 1)], Rim[(OR_MAXL + 1) * (OR_MAXL + 1)];
    double r2 = x * x + y * y + z * z;
    double r = sqrt(r2);
    /* R[l*L1+m] */
    Rre[0] = 1.0; Rim[0] = 0.0;
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) {
            double pr = Rre[(m - 1) * L1 + m - 1], pi = Rim[(m - 1) * L1 + m - 1];
            double f = -(2.0 * m - 1.0);
            Rre[m * L1 + m] = f * (x * pr - y * pi);
            Rim[m * L1 + m] = f * (x * pi + y * pr);
        }
        if (m + 1 <= lmax) {
            Rre[(m + 1) * L1 + m] = (2.0 * m + 1.0) * z * Rre[m * L1 + m];
            Rim[(m + 1) * L1 + m] = (2.0 * m + 1.0) * z * Rim[m * L1 + m];
        }
        for (int l = m + 2; l <= lmax; ++l) {
            Rre[l * L1 + m] = ((2.0 * l - 1.0) * z * Rre[(l - 1) * L1 + m] - (l + m - 1.0) * r2 * Rre[(l - 2) * L1 + m]) / (l - m);
            Rim[l * L1 + m] = ((2.0 * l - 1.0) * z * Rim[(l - 1) * L1 + m] - (l + m - 1.0) * r2 * Rim[(l - 2) * L1 + m]) / (l - m);
        }
    }
    double U = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int l = 0; l <= lmax; ++l) {
        double p = pow(r, -(2.0 * l + 1.0));          /* r^-(2l+1) */
        double q = (2.0 * l + 1.0) * p / r2;           /* -d(r^-(2l+1))/dx = q x */
        for (int m = 0; m <= l; ++m) {
            double c = (m == 0 ? 1.0 : 2.0) * factorial(l - m) / factorial(l + m);
            int jc = lm_index(l, m, 0);
            double Ac = Ar[jc], Bc = Br[jc], As = 0.0, Bs = 0.0;
            if (m > 0) { int js = lm_index(l, m, 1); As = Ar[js]; Bs = Br[js]; }
            double re = Rre[l * L1 + m], im = Rim[l * L1 + m];
            double ac = Ac * p + Bc, as = As * p + Bs;
            U += c * (re * ac + im * as);
            /* gradient of R_lm: components (dre, dim) for x, y, z */
            double dxr = 0, dxi = 0, dyr = 0, dyi = 0, dzr = 0, dzi = 0;
            if (l >= 1) {
                double upr = 0, upi = 0;   /* R_(l-1)(m+1) */
                if (m + 1 <= l - 1) { upr = Rre[(l - 1) * L1 + m + 1]; upi = Rim[(l - 1) * L1 + m + 1]; }
                if (m == 0) {
                    dxr = upr; dyr = upi;   /* d/dx R_l0 = Re(d+ R), d/dy R_l0 = Im(d+ R) */
                } else {
                    double f = -(double)(l + m) * (l + m - 1.0);
                    double dnr = 0, dni = 0;   /* f R_(l-1)(m-1) */
                    if (m - 1 <= l - 1) { dnr = f * Rre[(l - 1) * L1 + m - 1]; dni = f * Rim[(l - 1) * L1 + m - 1]; }
                    /* d/dx = (d+ + d-)/2, d/dy = (d+ - d-)/(2i) */
                    dxr = 0.5 * (upr + dnr); dxi = 0.5 * (upi + dni);
                    dyr = 0.5 * (upi - dni); dyi = -0.5 * (upr - dnr);
                }
                if (m <= l - 1) { dzr = (l + m) * Rre[(l - 1) * L1 + m]; dzi = (l + m) * Rim[(l - 1) * L1 + m]; }
            }
            double t = re * Ac + im * As;
            gx += c * (dxr * ac + dxi * as - q * x * t);
            gy += c * (dyr * ac + dyi * as - q * y * t);
            gz += c * (dzr * ac + dzi * as - q * z * t);
        }
    }
    *phi = -G * U;
    *ax = G * gx;
    *ay = G * gy;
    *az = G * gz;
}

/* Evaluate the node-interpolated expansion at one point (radius clamped). */
void or_mp_eval(const or_pot *p, const double *A, const double *B,
                double x, double y, double z, double *phi, double *ax, double *ay, double *az) {
    int lmax = p->lmax, nn = p->nnode, nlm = (lmax + 1) * (lmax + 1);
    double r = sqrt(x * x + y * y + z * z);
    double rc = r < p->rmin ? p->rmin : (r > p->rmax ? p->rmax : r);
    if (r > 0 && rc != r) { x *= rc / r; y *= rc / r; z *= rc / r; }
    if (!(r > 0)) { x = 0.0; y = 0.0; z = rc; }
    double lr0 = log(p->rmin), dl = (log(p->rmax) - lr0) / (nn - 1);
    int k = (int)floor((log(rc) - lr0) / dl);
    if (k < 0) k = 0;
    if (k > nn - 2) k = nn - 2;
    while (k > 0 && rc < exp(lr0 + k * dl)) --k;
    while (k < nn - 2 && rc >= exp(lr0 + (k + 1) * dl)) ++k;
    double t = (log(rc) - (lr0 + k * dl)) / dl;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double Ar[(OR_MAXL + 1) * (OR_MAXL + 1)], Br[(OR_MAXL + 1) * (OR_MAXL + 1)];
    for (int j = 0; j < nlm; ++j) {
        Ar[j] = A[(size_t)k * nlm + j] + t * (A[(size_t)(k + 1) * nlm + j] - A[(size_t)k * nlm + j]);
        Br[j] = B[(size_t)k * nlm + j] + t * (B[(size_t)(k + 1) * nlm + j] - B[(size_t)k * nlm + j]);
    }
    mp_field(lmax, p->G, x, y, z, Ar, Br, phi, ax, ay, az);
}

/* Exact truncated expansion at a point: A, B summed directly over the particles
 * at the point's own radius (no nodes, no interpolation). */
void or_mp_exact(const or_pot *p, int64_t N, const double *x, const double *y, const double *z,
                 const double *w, double px, double py, double pz,
                 double *phi, double *ax, double *ay, double *az) {
    int lmax = p->lmax, nlm = (lmax + 1) * (lmax + 1);
    double r = sqrt(px * px + py * py + pz * pz);
    double Ar[(OR_MAXL + 1) * (OR_MAXL + 1)] = {0}, Br[(OR_MAXL + 1) * (OR_MAXL + 1)] = {0};
    double Y[(OR_MAXL + 1) * (OR_MAXL + 1)];
    for (int64_t i = 0; i < N; ++i) {
        double ri = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
        angular(lmax, x[i], y[i], z[i], Y);
        double m = w[i] * p->Mtot;
        for (int l = 0; l <= lmax; ++l)
            for (int j = l * l; j < (l + 1) * (l + 1); ++j) {
                if (ri < r) Ar[j] += m * pow(ri, l) * Y[j];
                else Br[j] += m * pow(ri, -(l + 1)) * Y[j];
            }
    }
    (void)nlm;
    mp_field(lmax, p->G, px, py, pz, Ar, Br, phi, ax, ay, az);
}

/* Potential and acceleration of any supported kind at one point. */
static void field(const or_pot *p, const double *A, const double *B, double x, double y, double z,
                  double *phi, double *ax, double *ay, double *az) {
    if (p->kind == OR_POT_MULTIPOLE) or_mp_eval(p, A, B, x, y, z, phi, ax, ay, az);
    else or_potential(p, x, y, z, phi, ax, ay, az);
}

/* ------------------------------------------------------------------ observe */
void or_observe(const or_cfg *c, int64_t N, const double *x, const double *y, const double *z,
                const double *vx, const double *vy, const double *vz, const double *w,
                double *yout) {
    int J = c->J, T = nthreads();
    double *part = (double *)calloc((size_t)T * J, sizeof(double));
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int32_t jj[3 * OR_MAXBIN];
        double K[3 * OR_MAXBIN];
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            int n = or_kernel(&c->lay, x[i], y[i], z[i], vx[i], vy[i], vz[i], jj, K);
            for (int e = 0; e < n; ++e) part[(size_t)t * J + jj[e]] += w[i] * K[e];
        }
    }
    for (int j = 0; j < J; ++j) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += part[(size_t)t * J + j];
        yout[j] = s;
    }
    free(part);
}

/* ------------------------------------------------------------------ tracers */
static int binning_nbins(const or_layout *L, int b) {
    return L->kind[b] == OR_BIN_GRID ? L->nx[b] * L->ny[b] : L->nedge[b] - 1;
}

static double normal_density(double v, double mean, double s) {
    double d = (v - mean) / s;
    return exp(-0.5 * d * d) / (sqrt(2.0 * M_PI) * s);
}

/* Tracers grouped by bin: first[b] .. first[b+1] index into order[]. */
static void tracer_lists(const or_cfg *c, int nb, int32_t *first, int32_t *order) {
    const or_tracers *T = &c->trc;
    for (int b = 0; b <= nb; ++b) first[b] = 0;
    for (int t = 0; t < T->n; ++t) first[T->bin[t] + 1] += 1;
    for (int b = 0; b < nb; ++b) first[b + 1] += first[b];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    memcpy(fill, first, sizeof(int32_t) * (size_t)(nb + 1));
    for (int t = 0; t < T->n; ++t) order[fill[T->bin[t]]++] = t;
    free(fill);
}

/* L_t and M_b of the particles (see the header). */
void or_tracer_observe(const or_cfg *c, int64_t N, const double *x, const double *y, const double *z,
                       const double *vx, const double *vy, const double *vz, const double *w,
                       double *L, double *M) {
    const or_tracers *T = &c->trc;
    const or_layout *Ly = &c->lay;
    int nb = binning_nbins(Ly, T->binning);
    int32_t *first = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T->n > 0 ? T->n : 1));
    tracer_lists(c, nb, first, order);
    double ci = cos(Ly->incl), si = sin(Ly->incl);
    for (int t = 0; t < T->n; ++t) L[t] = 0.0;
    for (int b = 0; b < nb; ++b) M[b] = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int b = bin_of(Ly, T->binning, ci, si, x[i], y[i], z[i]);
        if (b < 0) continue;
        double vl = vy[i] * si + vz[i] * ci;
        M[b] += w[i];
        for (int e = first[b]; e < first[b + 1]; ++e) {
            int t = order[e];
            L[t] += w[i] * normal_density(vl, T->v[t], T->s[t]);
        }
    }
    free(first); free(order);
}

/* Leapfrog kick-drift-kick over dt (reading of "evolved in the potential"). */
static void push(const or_pot *p, const double *A, const double *B, double dt,
                 double *x, double *y, double *z, double *vx, double *vy, double *vz) {
    double phi, ax, ay, az;
    field(p, A, B, *x, *y, *z, &phi, &ax, &ay, &az);
    *vx += 0.5 * dt * ax; *vy += 0.5 * dt * ay; *vz += 0.5 * dt * az;
    *x += dt * *vx; *y += dt * *vy; *z += dt * *vz;
    field(p, A, B, *x, *y, *z, &phi, &ax, &ay, &az);
    *vx += 0.5 * dt * ax; *vy += 0.5 * dt * ay; *vz += 0.5 * dt * az;
}

/* Leapfrog only (no weights): n steps of the particles in a fixed analytic potential. */
void or_leapfrog(const or_pot *p, int64_t N, int64_t nsteps, double dt,
                 double *x, double *y, double *z, double *vx, double *vy, double *vz) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t s = 0; s < nsteps; ++s)
            push(p, NULL, NULL, dt, &x[i], &y[i], &z[i], &vx[i], &vy[i], &vz[i]);
}

/* Potential and acceleration for many points (analytic or node multipole). */
void or_field_many(const or_pot *p, const double *A, const double *B, int64_t N,
                   const double *x, const double *y, const double *z,
                   double *phi, double *ax, double *ay, double *az) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) field(p, A, B, x[i], y[i], z[i], &phi[i], &ax[i], &ay[i], &az[i]);
}

/* ------------------------------------------------------------------- a step */
int or_step(const or_cfg *c, or_state *s) {
    int64_t N = c->N;
    int J = c->J;
    const or_prior *P = &c->prior;
    /* 1 observe */
    or_observe(c, N, s->x, s->y, s->z, s->vx, s->vy, s->vz, s->w, s->yobs);
    /* 2 smooth (the smoothed vector starts at y(0)) */
    double g = c->dt / c->tau;
    for (int j = 0; j < J; ++j)
        s->ys[j] = s->n == 0 ? s->yobs[j] : s->ys[j] + g * (s->yobs[j] - s->ys[j]);
    /* 3 deviate */
    double chi2 = 0.0, chi2i = 0.0;
    for (int j = 0; j < J; ++j) {
        s->delta[j] = (s->ys[j] - c->Y[j]) / c->sigma[j];
        chi2 += s->delta[j] * s->delta[j];
        double di = (s->yobs[j] - c->Y[j]) / c->sigma[j];
        chi2i += di * di;
    }
    s->chi2 = chi2; s->chi2_inst = chi2i;
    /* 1-3 for the tracers */
    const or_tracers *T = &c->trc;
    int tnb = T->n > 0 ? binning_nbins(&c->lay, T->binning) : 0;
    int32_t *tfirst = NULL, *torder = NULL;
    if (T->n > 0) {
        or_tracer_observe(c, N, s->x, s->y, s->z, s->vx, s->vy, s->vz, s->w, s->tLobs, s->tMobs);
        for (int t = 0; t < T->n; ++t)
            s->tL[t] = s->n == 0 ? s->tLobs[t] : s->tL[t] + g * (s->tLobs[t] - s->tL[t]);
        for (int b = 0; b < tnb; ++b)
            s->tM[b] = s->n == 0 ? s->tMobs[b] : s->tM[b] + g * (s->tMobs[b] - s->tM[b]);
        double ll = 0.0;
        for (int t = 0; t < T->n; ++t) ll += log(s->tL[t] / s->tM[T->bin[t]]);
        s->loglike = ll;
        tfirst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tnb + 1));
        torder = (int32_t *)malloc(sizeof(int32_t) * (size_t)T->n);
        tracer_lists(c, tnb, tfirst, torder);
    }
    /* 4 prior */
    if (P->kind == OR_PRIOR_FLAT) {
        for (int64_t i = 0; i < N; ++i) s->what[i] = P->flat_value;
    } else if (P->kind == OR_PRIOR_HIST && s->n % P->period == 0) {
        int64_t nc = or_ncell(P);
        double *cs = (double *)malloc(sizeof(double) * (size_t)nc);
        double *cn = (double *)malloc(sizeof(double) * (size_t)nc);
        or_prior_means(P, N, s->x, s->y, s->z, s->vx, s->vy, s->vz, s->w, s->what, cs, cn);
        free(cs); free(cn);
    }
    /* 5 entropy and weight statistics */
    double S = 0.0, sw = 0.0, sw2 = 0.0, mw = INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        S -= s->w[i] * log(s->w[i] / s->what[i]);
        sw += s->w[i]; sw2 += s->w[i] * s->w[i];
        if (s->w[i] < mw) mw = s->w[i];
    }
    s->S = S; s->F = -0.5 * chi2 + c->mu * S;
    s->sumw = sw; s->sumw2 = sw2; s->minw = mw;
    /* 6 update */
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < N; ++i) {
        int32_t jj[3 * OR_MAXBIN];
        double K[3 * OR_MAXBIN];
        int n = or_kernel(&c->lay, s->x[i], s->y[i], s->z[i], s->vx[i], s->vy[i], s->vz[i], jj, K);
        double chi_term = 0.0;
        for (int e = 0; e < n; ++e) chi_term += K[e] * s->delta[jj[e]] / c->sigma[jj[e]];
        double G = -chi_term - c->mu * (log(s->w[i] / s->what[i]) + 1.0);
        if (T->n > 0) {
            int b = bin_of(&c->lay, T->binning, cos(c->lay.incl), sin(c->lay.incl), s->x[i], s->y[i], s->z[i]);
            if (b >= 0) {
                double vl = s->vy[i] * sin(c->lay.incl) + s->vz[i] * cos(c->lay.incl);
                double lt = 0.0;
                for (int e = tfirst[b]; e < tfirst[b + 1]; ++e) {
                    int t = torder[e];
                    lt += normal_density(vl, T->v[t], T->s[t]) / s->tL[t];
                }
                G += T->lambda * (lt - (tfirst[b + 1] - tfirst[b]) / s->tM[b]);
            }
        }
        double wn = c->update == 1 ? s->w[i] * exp(c->eps * c->dt * G)
                                   : s->w[i] * (1.0 + c->eps * c->dt * G);
        if (!isfinite(wn)) bad |= 2;
        else if (wn <= 0.0) bad |= 1;
        s->w[i] = wn;
    }
    free(tfirst); free(torder);
    if (bad) {
        s->status = (bad & 2) ? OR_NONFINITE : OR_NONPOSITIVE;
        s->bad_step = s->n;
        return s->status;
    }
    /* 7 push (self-consistent form: coefficients rebuilt after the drift, before
       the second kick, from the new positions and weights) */
    if (c->frozen) {
        /* particles held fixed */
    } else if (c->pot.kind == OR_POT_MULTIPOLE) {
        const or_pot *p = &c->pot;
        double dt = c->dt;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            double phi, ax, ay, az;
            field(p, s->mpA, s->mpB, s->x[i], s->y[i], s->z[i], &phi, &ax, &ay, &az);
            s->vx[i] += 0.5 * dt * ax; s->vy[i] += 0.5 * dt * ay; s->vz[i] += 0.5 * dt * az;
            s->x[i] += dt * s->vx[i]; s->y[i] += dt * s->vy[i]; s->z[i] += dt * s->vz[i];
        }
        or_mp_coeffs(p, N, s->x, s->y, s->z, s->w, s->mpA, s->mpB);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            double phi, ax, ay, az;
            field(p, s->mpA, s->mpB, s->x[i], s->y[i], s->z[i], &phi, &ax, &ay, &az);
            s->vx[i] += 0.5 * dt * ax; s->vy[i] += 0.5 * dt * ay; s->vz[i] += 0.5 * dt * az;
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i)
            push(&c->pot, NULL, NULL, c->dt, &s->x[i], &s->y[i], &s->z[i], &s->vx[i], &s->vy[i], &s->vz[i]);
    }
    s->n += 1;
    return OR_OK;
}

/* n steps; per-step statistics rows of 8 doubles:
 * chi2, chi2_inst, S, F, sum w, min w, sum w^2, step index. */
int or_run(const or_cfg *c, or_state *s, int64_t nsteps, double *stats) {
    for (int64_t k = 0; k < nsteps; ++k) {
        int rc = or_step(c, s);
        if (stats) {
            double *r = stats + 8 * k;
            r[0] = s->chi2; r[1] = s->chi2_inst; r[2] = s->S; r[3] = s->F;
            r[4] = s->sumw; r[5] = s->minw; r[6] = s->sumw2; r[7] = (double)(s->n - (rc == OR_OK));
        }
        if (rc != OR_OK) return rc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------ Philox4x32-10
 * Counter-based generator of Salmon, Moraes, Dror & Shaw (SC'11, "Parallel random
 * numbers: as easy as 1, 2, 3"): ten rounds of two 32x32->64 multiplies with the
 * published multipliers, key bumped by the published Weyl constants. */
void or_philox4x32(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Training-subset indices for prior refresh number `refresh`: index k uses
 * counter (k/4, refresh, 0, 0) under key (seed, 0) and word k%4, mapped to
 * [0, N) by the high word of a 32x32 product. */
void or_subset(uint32_t seed, uint32_t refresh, int64_t count, uint32_t N, int64_t *idx) {
    uint32_t key[2] = {seed, 0u};
    for (int64_t k = 0; k < count; k += 4) {
        uint32_t ctr[4] = {(uint32_t)(k / 4), refresh, 0u, 0u}, o[4];
        or_philox4x32(ctr, key, o);
        for (int e = 0; e < 4 && k + e < count; ++e)
            idx[k + e] = (int64_t)(((uint64_t)o[e] * N) >> 32);
    }
}
