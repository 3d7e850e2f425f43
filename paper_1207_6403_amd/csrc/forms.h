// forms.h -- arguments and launchers of the self-consistent multipole model,
// the learned prior and the stand-alone prior-cell kernel (the fused step
// kernel's own interface is in runtime.h).
#pragma once
#include "runtime.h"

namespace m2m {

// Self-consistent multipole potential (multipole.hip): node tables, interval
// sums and the particles the coefficient and kick kernels read.
// multipole tables always hold l <= kMpL: kMpNlm coefficients per node and kind
constexpr int kMpL = 8;
constexpr int kMpNlm = (kMpL + 1) * (kMpL + 1);
constexpr int kMpW = 2 * kMpNlm;   // A then B
constexpr int kMpMaxNodes = 512;
// FP32 node table: per node, per (l, m >= 0) one 16-byte entry (A cos, B cos,
// A sin, B sin; the sin pair zero for m = 0), rows l in order
constexpr int kMpRowF = 4 * (kMpL + 1) * (kMpL + 2) / 2;
// FP32 coefficient build: particles per lane of one accumulation chunk, and the
// particles of a chunk (one wave's work; all in one radial interval)
constexpr int kMpLaneRun = 16;
constexpr int kMpChunk = 64 * kMpLaneRun;
constexpr int kMpSortThreads = 1024;

template <typename T>
struct MpArgs {
    int32_t lmax, nn, nlm, nblock;   // nlm = (lmax + 1)^2 (readback tables); nblock: blocks of the plan
    T lr0, idl;                      // ln rmin, 1 / node spacing in ln r
    T rmin, rmax, G, Mtot, hdt;
    double lr0d, dld;                // ln rmin and node spacing in FP64 (interval decisions)
    const T* tab;                    // FP64: nn x 162 (A then B, l <= 8); FP32: nn x kMpRowF entries (read by the kicks)
    T* tab_out;                      // the same, written by the scan
    const double* rk;                // nn node radii (FP64)
    // FP32 coefficient build: the particles are counting-sorted by interval into
    // `sorted` (x, y, z, w) and summed chunk by chunk (kMpChunk particles of one
    // interval per wave) into per-chunk partials, then per interval in FP64
    int64_t n;                       // particles
    int32_t G_sort;                  // blocks of the interval count and scatter kernels
    int64_t R;                       // particles per such block (a multiple of kMpSortThreads)
    int32_t maxchunk;                // upper bound of the chunks: ceil(n / kMpChunk) + nn + 1
    uint16_t* key;                   // n: interval + 1 of each particle
    uint32_t* counts;                // (nn + 1) x G particles per interval and block
    uint32_t* offs;                  // (nn + 1) x G first sorted position of (interval, block) within the interval
    uint32_t* total;                 // nn + 1 particles per interval
    float4* sorted;                  // n
    float* part;                     // maxchunk x 162 chunk partials
    double* S;                       // (nn + 1) x 162 interval sums (interval -1 first)
    double* A64;                     // nn x nlm
    double* B64;                     // nn x nlm
    const T* src;                    // state buffer the coefficient and kick kernels work on
    int64_t stride;
    // accelerations (3 rows of `stride`) of the state the step starts from, read
    // by its first kick, and of the state it makes, written by the second kick
    // (the same field at the same points with the same node table)
    const T* acc_in;
    T* acc_out;
    int32_t kick;                    // launch_mp_build: 0 no kick, 1 kick and store, 2 store only
    const int32_t* block_tile0;
    const int64_t* tile_p0;
    const int32_t* tile_cnt;
    const int* flag;
};

struct MpLds {
    size_t kick_drift, coeff, kick;
};

// Learned prior (FP32 contexts, one model): network 3 -> 64 -> 64 -> 1 with tanh
// hidden units, parameters W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3.
constexpr int kMlpH = 64;
constexpr int kMlpNP = kMlpH * 3 + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;   // 4481
constexpr int kMlpW1 = 0, kMlpB1 = kMlpW1 + kMlpH * 3, kMlpW2 = kMlpB1 + kMlpH, kMlpB2 = kMlpW2 + kMlpH * kMlpH,
              kMlpW3 = kMlpB2 + kMlpH, kMlpB3 = kMlpW3 + kMlpH;
constexpr int kMlpSamples = 32;        // samples per training block
constexpr int kMlpTPS = 16;            // threads per sample
constexpr int kMlpTrainThreads = kMlpSamples * kMlpTPS;
constexpr int kMlpInferThreads = 256;
constexpr int kMlpMaxInferBlocks = 2048;

struct MlpArgs {
    const float* state;        // state buffer of the refresh step (rows x y z vx vy vz w, then tags)
    int64_t stride, n;
    const Exact* ex;           // FP64 potential, circular-orbit and seed tables
    float lcE0, lcEinv;        // origin and inverse spacing of the seed table
    double Emin, Emax;         // the prior's energy range
    uint32_t seed, q;          // sample generator key word and refresh index
    int32_t subset, batch;
    float4* sub;               // subset: (u0, u1, u2, ln w) per sample
    float* theta;              // kMlpNP parameters
    float* adam_m;
    float* adam_v;
    float* gpart;              // (batch / kMlpSamples) x kMlpNP partial gradients
    float lr, beta1, beta2, adam_eps;
    double fallback;
    float* what;               // n priors
    const float* cellmean;     // histogram prior cell means
    int32_t cellrow;           // tag row of the prior cell
    int32_t nblk;              // blocks of the inference passes (<= kMlpMaxInferBlocks)
    double* red;               // nblk x 2 per-block partials
    double* stats;             // gmax, sum w, sum e, judge numerator, judge, fallback used, refreshes
    float* loss;               // per sample (g - t)^2 / batch, or null
    int32_t mfma;              // 1: hidden-layer contractions on the matrix cores (BF16 operands, FP32 sums)
    // with mfma, for an analytic potential: the inference's features in FP32
    // (FP32 potential and the uniform-E Lc table), else from FP64 integrals
    const Pot<float>* pot32;   // null: FP64 features
    const float2* lcetab;      // kLcE (ln Lc, bound) pairs
    const int* flag;
};

// Prior cells of the state a.out (tags, and cell sums and counts into the cell
// columns of the partial slots) when the fused kernel observes without them.
hipError_t launch_cells(const StepArgs<float, float>& a, int pot_kind, int blocks, size_t lds, hipStream_t s);
hipError_t set_cells_lds_limit(size_t lds);

// One refresh of the learned prior: sample, nbatch Adam steps from step t0 + 1
// on, priors of every particle, judge and fallback.
hipError_t launch_mlp_refresh(const MlpArgs& a, int pot_kind, int t0, hipStream_t s);
// Loss terms and gradient of the mean squared error over the a.batch samples in
// a.sub at the parameters a.theta (the training kernels of a refresh, without
// the Adam step): grad gets kMlpNP values.
hipError_t launch_mlp_grad(const MlpArgs& a, float* grad, hipStream_t s);
// The same with no allocation: the partial rows and loss terms of at most
// kMlpNoAllocMax samples live in the library's static scratch array of the
// device (scratch_ptr, from mlp_noalloc_scratch); a.theta, a.sub and grad are
// the caller's device buffers; loss (device, nullable) gets the sum of the loss
// terms.  Calls that overlap on one device share the scratch and race.
constexpr int kMlpNoAllocMax = 8192;
constexpr size_t kMlpNoAllocFloats = (size_t)(kMlpNoAllocMax / kMlpSamples) * kMlpNP + kMlpNoAllocMax;
constexpr int kMaxDevices = 64;
hipError_t launch_mlp_grad_noalloc(MlpArgs a, float* scratch_ptr, float* grad, double* loss, hipStream_t s);
// Device address of that scratch array on `device` (which must be current),
// looked up once per device and kept.
hipError_t mlp_noalloc_scratch(int device, float** out);

// Weight update, first kick and drift of a multipole step (the coefficients of
// the new state and the second kick follow with launch_mp_build).
template <typename T, typename PT>
hipError_t launch_mp_step(const StepArgs<T, PT>& a, const MpArgs<T>& mp, uint64_t sig, int nbin, int blocks,
                          const MpLds& lds, hipStream_t s);
// Coefficients of the particles in mp.src, then per mp.kick: nothing (0), the
// second kick with its accelerations stored in mp.acc_out (1), or only the
// accelerations (2: the initial state's, for the first step's first kick).
// ek0/ek1 (nullable): events recorded around the kick kernel.
template <typename T>
hipError_t launch_mp_build(const MpArgs<T>& mp, int blocks, const MpLds& lds, hipStream_t s,
                           hipEvent_t ek0 = nullptr, hipEvent_t ek1 = nullptr);
template <typename T, typename PT>
hipError_t set_mp_lds_limit(size_t lds);

// Velocity second moments in spherical shells of the particles [p0, p1) of a
// state buffer (moments.hip): per block, nshell sums each of w, w v_r^2,
// w v_theta^2 and w v_phi^2 into its row of `part` (blocks x 4 nshell), then
// their sum in block order into `out` (device, 4 x nshell).
constexpr int kShellThreads = 256;
constexpr int kShellMax = 256;
constexpr int kShellBlocks = 512;
template <typename T>
struct ShellArgs {
    const T* state;
    int64_t stride, p0, p1;
    const double* edges;   // nshell + 1 increasing radii
    int32_t nshell;
    double* part;
};
template <typename T>
hipError_t launch_shell_moments(const ShellArgs<T>& a, int blocks, double* out, hipStream_t s);

// Discrete tracers (tracers.hip): tracers grouped by bin (first[b] .. first[b+1]),
// each with its velocity V, inverse width is = 1/s and density factor
// nf = 1/(sqrt(2 pi) s); per tracer the smoothed sum Ls and the update factor
// cL = lambda / Ls, per bin the smoothed mass Ms and cM = -lambda n_b / Ms.
constexpr int kTrcBlocks = 256;
template <typename T>
struct TracerArgs {
    const T* state;          // state buffer (value rows, then tag rows)
    int64_t stride, n;
    int32_t tagrow;          // tag row of the tracers' binning
    int32_t ntr, nb;
    T sini, cosi;
    const int32_t* first;    // nb + 1
    const T* V;
    const T* is;
    const T* nf;
    const T* cL;             // ntr
    const T* cM;             // nb
    T* extra;                // n: the likelihood's term of G (tracer_grad)
    double* part;            // blocks x (ntr + nb) partial sums (tracer_observe)
    int32_t nblk;            // blocks of tracer_observe
    double* Ls;              // ntr smoothed sums
    double* Ms;              // nb smoothed masses
    T* cL_out;
    T* cM_out;
    double* loglike;
    const int32_t* tbin;     // ntr: bin of each tracer (CSR order)
    double g;                // dt / tau
    double lambda;
    int32_t first_obs;       // 1: the smoothed sums start at this observation
    const int* flag;
};
// Sums L_t, M_b of the state (per-block partials), then their smoothing and the
// update factors.
template <typename T>
hipError_t launch_tracer_observe(const TracerArgs<T>& a, hipStream_t s);
// The log-likelihood of the smoothed sums into *loglike.
template <typename T>
hipError_t launch_tracer_loglike(const TracerArgs<T>& a, hipStream_t s);
// extra[p] of every particle of the state.
template <typename T>
hipError_t launch_tracer_grad(const TracerArgs<T>& a, hipStream_t s);
// Dynamic LDS the tracer kernels need, and the attribute that allows it.
template <typename T>
size_t tracer_lds(const TracerArgs<T>& a);
template <typename T>
hipError_t set_tracer_lds_limit(size_t lds);

}  // namespace m2m
