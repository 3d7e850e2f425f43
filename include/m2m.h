/*
 * m2m.h -- C ABI of the MI355X (gfx950) library for the per-timestep loop of the
 * NMAGIC made-to-measure (M2M) particle method (Morganti & Gerhard,
 * "NMAGIC made-to-measure particle models of galaxies").
 *
 * Problem statement (section 2 of the paper): an N-body system of particles with
 * weights w_i is evolved in a gravitational potential (fixed and known a priori,
 * or self-consistently computed from the particles) while the weights are
 * adapted to maximise the merit function F = -chi^2/2 + mu S (eq. 1), where
 * chi^2 measures the deviations between target and model observables and
 * S = -sum_i w_i ln(w_i / what_i) is a pseudo-entropy (eq. 2) that pushes the
 * weights towards priors what_i.  Priors are flat (what_i = 1/N, section 2.1)
 * or moving: recomputed from the weight distribution over integrals of motion
 * (section 2.1).
 *
 * One library step n (all on the GPU, no host round trip):
 *   G_i = -sum_j K_j(z_i) Dt_j/sigma_j - mu (ln(w_i/what_i) + 1)
 *   w_i <- w_i exp(eps dt G_i)            (or w_i (1 + eps dt G_i), see update)
 *   z_i <- kick-drift-kick leapfrog over dt
 *   y_j  = sum_i w_i K_j(z_i)              (observables of the new state)
 *   ys_j <- ys_j + (dt/tau) (y_j - ys_j)   (temporal smoothing)
 *   Dt_j = (ys_j - Y_j)/sigma_j,  chi^2 = sum_j Dt_j^2
 *   moving prior: what_i = mean weight of the particles in i's phase-space cell
 * The observable kernels K_j are linear in the weights: mass in 3D shells,
 * projected annuli or sky pixels, and the first/second line-of-sight velocity
 * moments sum w v_los, sum w v_los^2 in annuli or pixels.
 *
 * Conventions for every entry point:
 *  - Status codes only; nothing throws or aborts across this boundary.  After an
 *    error the context keeps a message (m2m_last_error).
 *  - A context is not thread-safe.  Calls on one context are ordered on its
 *    stream.  Separate contexts are independent.
 *  - The caller owns every buffer it passes.  m2m_create copies its inputs and
 *    keeps no caller pointer.  Readbacks synchronise the context's stream and
 *    then write the caller's buffer.
 *  - "device_ptrs"/"device_ptr" = 1 means the pointer is a device address on
 *    the context's device (for example torch.Tensor.data_ptr()); 0 means host.
 */
#ifndef M2M_H
#define M2M_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define M2M_ABI_VERSION 2
#define M2M_MAX_BINNINGS 4
#define M2M_MAX_EDGES 256
#define M2M_MLP_NPARAM 4481

typedef enum {
    M2M_OK = 0,
    M2M_ERR_INVALID = 1,            /* bad argument; nothing was changed                  */
    M2M_ERR_NOMEM = 2,              /* device allocation failed                           */
    M2M_ERR_DEVICE = 3,             /* a HIP call failed; the context should be destroyed */
    M2M_ERR_NONPOSITIVE_WEIGHT = 4, /* an update produced w <= 0; state is the last good step */
    M2M_ERR_NONFINITE = 5,          /* an update produced a non-finite weight; idem        */
    M2M_ERR_UNSUPPORTED = 6         /* valid request this build does not support           */
} m2m_status;

enum { M2M_F32 = 0, M2M_F64 = 1 };
enum { M2M_POT_HERNQUIST = 0, M2M_POT_LOG = 1, M2M_POT_HERNQUIST_NFW = 2, M2M_POT_MULTIPOLE = 3 };
enum { M2M_BIN_SHELL = 1, M2M_BIN_ANNULUS = 2, M2M_BIN_GRID = 3 };
/* Moment codes of a binning: mass, first and second line-of-sight moments, and
 * the Gauss-Hermite moments h1..h4 (section 1: absorption-line kinematics from
 * long-slit and integral-field spectra) of each bin's line-of-sight velocity
 * distribution expanded about the Gaussian (V_b, sigma_b) given with the data
 * (van der Marel & Franx 1993): kernel 2 sqrt(pi) alpha(nu) H_m(nu),
 * nu = (v_los - V_b)/sigma_b, alpha(nu) = exp(-nu^2/2)/sqrt(2 pi), H_m the
 * normalised Hermite polynomials; its mass-weighted sum over the particles of a
 * bin is the bin's mass times h_m. */
enum { M2M_MOM_MASS = 0, M2M_MOM_V = 1, M2M_MOM_V2 = 2, M2M_MOM_H1 = 3, M2M_MOM_H2 = 4, M2M_MOM_H3 = 5,
       M2M_MOM_H4 = 6 };
enum { M2M_PRIOR_FLAT = 0, M2M_PRIOR_HIST = 1, M2M_PRIOR_MLP = 2 };
enum { M2M_UPDATE_EULER = 0, M2M_UPDATE_EXP = 1 };

/* Gravitational potential of one model (section 2: fixed a priori, or
 * self-consistent).  Units are the caller's.
 *   HERNQUIST      Phi = -G M/(r + a)
 *   LOG            Phi = v0^2/2 ln(Rc^2 + x^2 + y^2 + z^2/q^2)
 *   HERNQUIST_NFW  Hernquist(G, M, a) - G Mh ln(1 + r/rs)/r
 *   MULTIPOLE      self-consistent multipole expansion to l <= lmax of the
 *                  particles (mass w_i * Mtot), coefficients at nnode
 *                  log-spaced radii in [rmin, rmax], linear in ln r between
 *                  them; radii outside the range are clamped.  Rebuilt every
 *                  step between the drift and the second kick.  One model per
 *                  context; FP32 contexts hold the node table in LDS, so
 *                  nnode is limited by it (720 bytes per node of the 160 KB:
 *                  at most 226 nodes; UNSUPPORTED beyond). */
typedef struct {
    int32_t kind;
    int32_t lmax, nnode, reserved;
    double G, M, a;
    double v0, Rc, q;
    double Mh, rs;
    double rmin, rmax, Mtot;
} m2m_potential;

/* One group of observation bins.  kind SHELL bins r = |x| and ANNULUS bins the
 * projected radius R = |(X, Y)| against nedge strictly increasing edges (bins
 * are [e_k, e_k+1)); GRID bins the sky plane into nx * ny pixels over
 * [x0, x1) x [y0, y1), pixel k = iy * nx + ix.  mom[0..nmom-1] lists the
 * moment codes fitted in these bins (M2M_MOM_*: 0 = mass, 1 = sum w v_los,
 * 2 = sum w v_los^2, 3..6 = Gauss-Hermite h1..h4); a binning that lists a
 * Gauss-Hermite code gives gh, 2 * nb values (host, copied at creation): V_b of
 * every bin, then sigma_b > 0 of every bin. */
typedef struct {
    int32_t kind;
    int32_t nmom;
    int32_t mom[3];
    int32_t nedge;
    const double *edges;     /* host, nedge values (SHELL, ANNULUS)     */
    int32_t nx, ny;
    double x0, x1, y0, y1;   /* GRID extent                             */
    const double *gh;        /* host, Gauss-Hermite V_b[nb], sigma_b[nb] */
} m2m_binning;

/* Observation layout.  Sky coordinates for inclination incl (radians):
 * X = x, Y = y cos(incl) - z sin(incl), v_los = vy sin(incl) + vz cos(incl).
 * Observable index j runs over binnings in order, then their moments in the
 * listed order, then bins; J is the total. */
typedef struct {
    double incl;
    int32_t nbin;
    int32_t reserved;
    m2m_binning bin[M2M_MAX_BINNINGS];
} m2m_obs_layout;

/* Priors what_i (section 2.1).  FLAT: constant flat_value (<= 0 means 1/N_m).
 * HIST: moving prior; what_i = mean weight of the particles in i's cell, cells
 * on n[0] uniform bins of E in [Emin, Emax] (clamped to the edge cells), then
 * n[1] bins of L/Lc(E) in [0, 1] (ax2 = 0) or Lz/Lc(E) in [-1, 1] (ax2 = 1), then
 * n[2] bins of Lz/L in [-1, 1] (n[2] = 1: unused); Lc(E) is the angular momentum
 * of the circular orbit of energy E.  Recomputed every `period` steps and held
 * per particle in between.  MLP: learned prior ln what = g(u) + c with g a
 * 3-64-64-1 tanh network of u = (2(E-Emin)/(Emax-Emin) - 1, 2 L/Lc - 1, Lz/L),
 * retrained every `period` steps on the current weights (Adam on the mean
 * squared error of g - ln w over a Philox4x32-10 sample of mlp_subset
 * particles in minibatches of mlp_batch), with the HIST prior on the same cells
 * as fallback whenever the w-weighted mean |ln what_mlp - ln what_hist| exceeds
 * `fallback`.  E and Lc are measured in `ref` (ref.kind < 0: the model's own
 * potential; required for MULTIPOLE models). */
typedef struct {
    int32_t kind;
    int32_t ax2;
    int32_t n[3];
    int32_t period;
    const double *Erange;    /* host, 2 * n_models (Emin, Emax), copied at creation;
                                or NULL: per model, min and max of E(0) over its
                                particles, computed in FP64 from the stored values */
    double flat_value;
    m2m_potential ref;
    int32_t mlp_subset, mlp_batch;
    double lr, beta1, beta2, adam_eps, fallback;
    uint32_t seed;
    int32_t mlp_mfma;        /* MLP: 1 = the hidden-layer contractions of the training
                                and of the inference over all particles on the matrix
                                cores (BF16 operands, FP32 accumulation; the inference
                                takes its features from FP32 integrals); 0 = FP32
                                throughout with FP64 features (the tight mode) */
    const float *mlp_init;   /* host, M2M_MLP_NPARAM initial parameters (MLP only) */
} m2m_prior;

/* Run configuration.  Models are independent M2M runs stepped together: model m
 * owns particles [model_offsets[m], model_offsets[m+1]) and potentials[m]; all
 * share the layout and prior settings.  update selects the integration of
 * dw/dt = eps w G over dt: EXP (w exp(eps dt G), default) or EULER
 * (w (1 + eps dt G)).  frozen = 1 keeps the particles fixed (weights still adapt). */
typedef struct {
    int32_t abi_version;       /* must be M2M_ABI_VERSION                 */
    int32_t precision;         /* M2M_F32 or M2M_F64 particle arithmetic  */
    int32_t update;
    int32_t frozen;
    double dt, eps, mu, tau;   /* dt > 0, eps >= 0, mu >= 0, tau >= dt    */
    int32_t n_models;          /* >= 1                                    */
    int32_t reserved;
    const int64_t *model_offsets;       /* host, n_models + 1, first 0     */
    const m2m_potential *potentials;    /* host, n_models                  */
    m2m_prior prior;
    void *stream;              /* hipStream_t to run on; NULL = default   */
} m2m_config;

/* Targets Y_j and errors sigma_j > 0 (FP64, host): J values shared by every
 * model (per_model = 0) or n_models * J values, model-major (per_model = 1). */
typedef struct {
    const double *Y;
    const double *sigma;
    int32_t J;
    int32_t per_model;
} m2m_target;

/* Per-step, per-model statistics: chi2 of the smoothed and of the instantaneous
 * observables, S (eq. 2), F (eq. 1), sum w, min w, sum w^2,
 * n_eff = (sum w)^2 / sum w^2, all of the state at the start of `step`. */
typedef struct {
    double chi2, chi2_inst, S, F, sum_w, min_w, sum_w2, n_eff;
    int64_t step;
    int32_t model;
    int32_t reserved;
} m2m_step_stats;

/* Launch shape of the fused step kernel (see m2m_autotune).  timing = 1 makes
 * m2m_step launch without graphs and time every fused step kernel (MULTIPOLE
 * models: the second-kick kernel, which evaluates the field) with HIP events
 * attached to its launch, which take the kernel's own start and end times
 * (read with m2m_kernel_time). */
typedef struct {
    int32_t threads;        /* 64..1024, multiple of 64 (FP64: at most 256) */
    int32_t ilp;            /* particles per thread per tile: 1 or 2        */
    int32_t blocks_per_cu;  /* blocks per compute unit (grid = CUs x this)  */
    int32_t graph_steps;    /* steps captured per HIP graph (0: none)       */
    int32_t timing;
    int32_t reserved;
} m2m_launch;

typedef struct m2m_ctx m2m_ctx;

int32_t m2m_abi_version(void);

/* Paper section 2 (the problem: an N-body particle model evolved in a given or
 * self-consistent potential whose weights are fitted to target observables with
 * errors) and section 2.1 (initial weights 1/N, flat or moving priors).
 * Create a context: validate, copy the particles (xv: 6 * N values, SoA
 * x[N] y[N] z[N] vx[N] vy[N] vz[N]; w: N values > 0, both in cfg precision),
 * observe the initial state (y(0), smoothed y = y(0), priors at step 0).
 * Errors: INVALID (w <= 0 or non-finite, J or model offsets inconsistent,
 * dt <= 0, mu < 0, eps < 0, tau < dt, edges not increasing, unknown kinds,
 * unsupported MULTIPOLE/MLP combinations), NOMEM, DEVICE.  *out is NULL on error. */
m2m_status m2m_create(const m2m_config *cfg, const m2m_obs_layout *layout,
                      const m2m_target *target, const void *xv, const void *w,
                      int32_t device_ptrs, m2m_ctx **out);

/* Paper section 2: the weights are adapted, by maximising F of eq. 1 with the
 * entropy of eq. 2, while the particles are evolved; section 2.1: the moving
 * priors are recomputed from the weight distribution as the run proceeds.
 * Advance n_steps >= 0 steps.  last (nullable) receives n_models rows: the
 * statistics of the final step taken.  On NONPOSITIVE_WEIGHT / NONFINITE the
 * context stays at the start of the failing step (whose index is in the
 * message and in m2m_step_index); later calls return the same error. */
m2m_status m2m_step(m2m_ctx *ctx, int64_t n_steps, m2m_step_stats *last);

/* Steps taken so far (host mirror of the device counter); -1 for a NULL ctx. */
int64_t m2m_step_index(const m2m_ctx *ctx);

/* Paper section 2: the model observables compared with the target data, their
 * deviations and chi^2 (the first term of eq. 1).
 * Observables of model m at the current state: y (last observe), y_smooth,
 * delta = (y_smooth - Y)/sigma (J values each, host, nullable, caller-owned)
 * and chi2 (nullable).  Synchronises the context's stream.  INVALID for a
 * model outside [0, n_models). */
m2m_status m2m_observables(m2m_ctx *ctx, int32_t model, double *y, double *y_smooth,
                           double *delta, double *chi2);

/* Paper section 2 (eq. 1 and 2): the particle weights w_i that the fit adapts.
 * Current weights, N values in cfg precision, into w_out (host, or device when
 * device_ptr = 1; caller-owned); synchronises the context's stream.  INVALID for
 * a null argument. */
m2m_status m2m_weights(m2m_ctx *ctx, void *w_out, int32_t device_ptr);

/* Paper section 2.1 (and eq. 2): the priors what_i of the entropy, flat or moving
 * (the mean weight over a cell of the integrals of motion, or the learned form).
 * Priors what_i the next step will use (N values, cfg precision, nullable;
 * MLP: those of the last refresh; host, or device when device_ptr = 1) and the
 * cell table (n_models * ncell FP64 cell means, host, nullable; HIST and MLP
 * only), both caller-owned.  Synchronises the context's stream.  INVALID when a
 * cell table is asked of a flat prior. */
m2m_status m2m_priors(m2m_ctx *ctx, void *what_out, double *cell_mean, int32_t device_ptr);

/* Paper section 2: the phase-space coordinates of the evolved particles (the
 * state a run can be restarted from with m2m_create, together with the weights).
 * Current particles, 6 * N values SoA (same layout as m2m_create), into xv_out
 * (host, or device when device_ptr = 1; caller-owned); synchronises the stream.
 * INVALID for a null argument. */
m2m_status m2m_particles(m2m_ctx *ctx, void *xv_out, int32_t device_ptr);

/* Decisions stored with the current state (section 2: the observables are
 * kernel sums over bins of the particles' coordinates; section 2.1: the moving
 * prior averages over cells of the integrals of motion).  out receives
 * (nbin + 1) * N uint16 values, row-major: row b < nbin holds each particle's
 * bin within binning b (grid pixel iy * nx + ix, or shell/annulus index; 0xFFFF
 * outside the binning), row nbin its prior cell ((iE * n1 + i2) * n2 + i3).
 * The cell row is defined when the moving prior took the cells of the current
 * state: always for a period of 1, else when the step index is a multiple of
 * the period; otherwise (and for a flat prior) its contents are unspecified.
 * Host or device memory (device_ptr), owned by the caller; synchronises the
 * context's stream.  M2M_ERR_INVALID for a null argument. */
m2m_status m2m_tags(m2m_ctx *ctx, uint16_t *out, int32_t device_ptr);

/* Statistics rows of the most recent steps, oldest first (ring of the last
 * 4096 steps per model).  out holds max_rows rows; *n_rows gets the count. */
m2m_status m2m_history(m2m_ctx *ctx, m2m_step_stats *out, int64_t max_rows, int64_t *n_rows);

/* Paper section 4: the data are fitted in a sequence of gravitational potentials
 * (here the n_models models of one context, each with its own potential) and
 * the fits are compared.  For the statistics of the last step taken: chi2
 * (n_models values, the smoothed chi^2 of each model), delta (n_models values,
 * chi2 - min over models) and *best (the model of least chi^2; the first on a
 * tie).  Host outputs, each nullable.  INVALID when no step has been taken. */
m2m_status m2m_delta_chi2(m2m_ctx *ctx, double *chi2, double *delta, int32_t *best);

/* Paper section 3, Fig. 1: the anisotropy profile a fit recovers for a
 * spherical target.  Velocity second moments of model `model`'s weighted
 * particles in the current state, in spherical shells [edges[k], edges[k+1])
 * of r = |x| about the origin: out (host, 4 * nshell FP64 values, row-major)
 * gets, per shell, sum w, sum w v_r^2, sum w v_theta^2 and sum w v_phi^2
 * (spherical components about the z axis; v_phi = 0 on the axis).  Particles
 * outside every shell add nothing.  Then beta(r) = 1 - (row 2 + row 3) /
 * (2 row 1).  edges: nshell + 1 strictly increasing finite radii, edges[0] > 0
 * (host, copied); 1 <= nshell <= M2M_SHELL_MAX.  Sums in FP64 on the GPU, in
 * a fixed block order (the order of additions inside a block varies, so the
 * last bits may differ between calls).  Synchronises the context's stream.
 * INVALID for a bad model index, edges or nshell. */
#define M2M_SHELL_MAX 256
m2m_status m2m_shell_moments(m2m_ctx *ctx, int32_t model, const double *edges, int32_t nshell, double *out);

/* Paper section 1 lists PNe velocities among the data: discrete tracers, each
 * with a sky position and one line-of-sight velocity.  Reading (the likelihood
 * term of NMAGIC's discrete-velocity fits): tracer t lies in bin b_t of one
 * layout binning (an annulus or sky-grid binning); its likelihood is the
 * model's line-of-sight velocity density at V_t in that bin,
 *   L_t = sum_i w_i [bin(z_i) = b_t] phi(v_los,i; V_t, s_t),  M_b = sum_i w_i [bin(z_i) = b],
 * both smoothed over time like the observables, and lambda sum_t ln(L_t / M_(b_t))
 * joins the merit function; the weight update gains its gradient
 *   lambda (sum_{t in b(z_i)} phi(v_los,i; V_t, s_t) / L_t - n_(b(z_i)) / M_(b(z_i)))
 * (phi the normal density of width s_t, n_b the tracers in bin b). */
typedef struct {
    int32_t binning;        /* index of the layout binning the tracers are binned in */
    int32_t n;              /* tracers, 1 .. M2M_TRACERS_MAX                          */
    const int32_t *bin;     /* n: the tracer's bin within that binning               */
    const double *v;        /* n: its line-of-sight velocity                         */
    const double *width;    /* n: kernel width s_t > 0 (velocity error and smoothing) */
    double lambda;          /* weight of the log-likelihood in the merit function    */
} m2m_tracers;
#define M2M_TRACERS_MAX 8192

/* Attach discrete tracers to a single-model context before its first step (a
 * fixed analytic potential; not with the learned prior).  Host arrays, copied.
 * Observes the tracers in the initial state (their smoothed sums start there).
 * INVALID for a bad binning index or bin, n outside [1, M2M_TRACERS_MAX], a
 * width <= 0, a non-finite value, a step already taken or tracers already set;
 * UNSUPPORTED for batched, multipole or learned-prior contexts. */
m2m_status m2m_set_tracers(m2m_ctx *ctx, const m2m_tracers *tracers);

/* The tracers' smoothed sums of the current state and their log-likelihood
 * sum_t ln(L_t / M_(b_t)): loglike (host scalar), L (n values, in the order the
 * tracers were given), M (the binning's bins); each nullable.  Synchronises the
 * context's stream.  INVALID without tracers. */
m2m_status m2m_tracer_state(m2m_ctx *ctx, double *loglike, double *L, double *M);

/* Node coefficients of a MULTIPOLE model (sections 1 and 2: the potential
 * computed from the particles), as used by the first kick of the next step:
 * A and B, nnode * (lmax+1)^2 FP64 values each (host; node k at k*(lmax+1)^2,
 * coefficient (l, m >= 0, cos) at l*l + 2m - 1 for m > 0, l*l for m = 0, the
 * sin part one after the cos part).  A(r_k) sums m_i r_i^l P_l^m e^(i m phi_i)
 * over the particles below node radius r_k, B(r_k) m_i r_i^-(l+1) P_l^m e^(i m
 * phi_i) over the rest.  FP32 contexts sum per-block FP32 partials in FP64.
 * INVALID when the model is not a multipole. */
m2m_status m2m_multipole_tables(m2m_ctx *ctx, double *A, double *B);

/* State of an MLP prior (section 2.1: priors over integrals of motion that
 * follow the weight distribution; here learned): theta gets the
 * M2M_MLP_NPARAM FP32 parameters as of the last refresh (W1[64][3], b1[64],
 * W2[64][64], b2[64], W3[64], b3), judge the w-weighted mean |ln what_mlp -
 * ln what_hist| of the last refresh, used_fallback whether it exceeded the
 * threshold (the histogram prior then applies until the next refresh),
 * refreshes the count so far.  Every output is a host pointer and nullable.
 * A refresh runs before the update of every step n with n % period == 0, on
 * that step's state.  INVALID when the prior is not MLP.  The learned prior
 * runs in FP32 contexts of one model (m2m_create: UNSUPPORTED otherwise);
 * mlp_batch must be a multiple of 32 and divide mlp_subset. */
m2m_status m2m_mlp_state(m2m_ctx *ctx, float *theta, double *judge, int32_t *used_fallback, int64_t *refreshes);

/* Loss and gradient of the MLP prior's training objective (the mean over n
 * samples of (g(u) - t)^2) at parameters theta, computed by the same GPU
 * kernels as a refresh's minibatches (FP32; the blocks' sums added in FP64).
 * theta: host, M2M_MLP_NPARAM values in the layout of m2m_mlp_state; samples:
 * host, n rows of (u0, u1, u2, t); n a positive multiple of 32.  grad (host,
 * M2M_MLP_NPARAM) gets the gradient, loss (host, nullable) the mean.  The
 * context's parameters and state are not touched; device scratch is allocated
 * for the call.  INVALID when the prior is not MLP. */
m2m_status m2m_mlp_loss_grad(m2m_ctx *ctx, const float *theta, const float *samples, int32_t n, float *grad,
                             double *loss);

/* The loss and gradient of m2m_mlp_loss_grad, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): this call allocates nothing.  Its working memory (the
 * training blocks' partial gradient rows and the per-sample loss terms) is a
 * static array of the library, one copy per device, sized for at most
 * M2M_MLP_NOALLOC_MAX samples (4.6 MB), held from the first m2m_create on that
 * device until the process ends.  theta (M2M_MLP_NPARAM FP32), samples (n rows
 * of (u0, u1, u2, t) FP32, 16-byte aligned), grad (M2M_MLP_NPARAM FP32) and loss
 * (one FP64, nullable: the sum of the per-sample terms, i.e. the mean) are
 * device pointers on the context's device, owned by the caller.  The work is
 * enqueued on the context's stream and the call returns without waiting:
 * results are valid once that stream has been synchronised.  The kernels are
 * those of m2m_mlp_loss_grad (bitwise the same gradient).  Every call on a
 * device shares that device's array: calls that overlap on one device (other
 * contexts, other streams) race.  INVALID for a null argument, a context
 * without a learned prior, n not a positive multiple of 32 or above
 * M2M_MLP_NOALLOC_MAX, or misaligned samples. */
#define M2M_MLP_NOALLOC_MAX 8192
m2m_status m2m_mlp_loss_grad_noalloc(m2m_ctx *ctx, const float *theta, const float *samples, int32_t n,
                                     float *grad, double *loss);

/* Time candidate launch shapes (threads x ilp x blocks_per_cu) on trial_steps
 * steps each, restore the state, keep the fastest; chosen may be NULL.  The
 * choice is cached in the JSON file named by $M2M_AUTOTUNE_CACHE if set. */
m2m_status m2m_autotune(m2m_ctx *ctx, int32_t trial_steps, m2m_launch *chosen);

/* Read or set the launch shape (graph_steps = 0 disables HIP graphs). */
m2m_status m2m_get_launch(const m2m_ctx *ctx, m2m_launch *out);
m2m_status m2m_set_launch(m2m_ctx *ctx, const m2m_launch *in);

/* Average duration in milliseconds of the fused step kernel (MULTIPOLE
 * models: of the second-kick kernel) over the last m2m_step call, from the HIP
 * events attached to its launches (0 if the call used graphs or took no steps);
 * *launches gets the launch count. */
m2m_status m2m_kernel_time(const m2m_ctx *ctx, double *ms_per_launch, int64_t *launches);

/* End of the run of section 2: free every device buffer of the context (NULL is
 * ignored); waits for the context's stream first. */
void m2m_destroy(m2m_ctx *ctx);

/* Error reporting of this boundary (no paper passage: status codes only cross
 * it).  Message of the last error on ctx ("" if none); with ctx NULL, the message
 * of the last failed m2m_create on this thread.  The string is owned by the
 * library and valid until the next call on the same context. */
const char *m2m_last_error(const m2m_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* M2M_H */
