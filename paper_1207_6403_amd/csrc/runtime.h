// runtime.h -- kernel argument blocks and launch helpers shared by the
// library's translation units (never exported through the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace m2m {

constexpr int kRing = 4096;          // statistics rows kept per model
constexpr int kSlotsPerSplit = 32;   // partial slots in flight per finalise thread
constexpr int kFinCols = 32;         // columns per finalise block
constexpr int kFinGroups = 8;        // slot groups per column (256 threads)

struct StatRow {
    double chi2, chi2_inst, S, F, sum_w, min_w, sum_w2, n_eff;
    long long step;
    int32_t model, reserved;
};

// Fused step: update + push + observe + prior cells (one particle pass).
template <typename T, typename PT>
struct StepArgs {
    // State buffers: 7 value rows (x y z vx vy vz w) then tag rows (bin of each
    // binning, prior cell), `stride` entries each; less than 4 GiB in all.
    const T* in;            // state at step n
    T* out;                 // state at step n+1 (the state at step n when observing only)
    int64_t stride;
    T* what;                // per-particle priors (stored modes)
    const int32_t* tile_model;
    const int64_t* tile_p0;
    const int32_t* tile_cnt;
    const int32_t* block_tile0;   // nblocks + 1
    const int32_t* block_slot0;   // first partial slot of each block
    const Pot<T>* pots;           // per model
    const T* lctab;               // kLcTab circular-orbit energies per model
    const float* lcetab;          // kLcE (Lc, error bound) pairs per model (FP32 path)
    const T* erange;              // 2 per model
    const T* flatw;               // per model
    const T* cvec;                // M * J: Dt_j / sigma_j
    const T* cellmean;            // M * NC
    PT* part;                     // partial slots, chunk-major per model
    const int64_t* slot_base;     // column j of slot q: part[slot_base[q] + (j / kFinCols) *
    const int32_t* slot_stride;   //   slot_stride[q] + j % kFinCols]
    double* seg_stats;            // nslot * 4
    const T* edges;
    int32_t nedge;
    int32_t pcols, jpad;
    Layout<T> lay;
    Cells cells;
    const Exact* ex;              // FP64 constants and tables (device memory)
    T dt, eps, mu;
    uint32_t flags;               // kObserve | kWhat* | kAccum | kExpLaw | kFrozen
    int32_t cellrow;              // tag row of the prior cell
    int* flag;
    long long* bad_step;
    const long long* d_step;
};

// Step flags.  kWhat: where the prior of the update comes from -- 0 flat,
// 1 cell-mean table, 2 table and store it per particle, 3 the stored priors.
constexpr uint32_t kObserve = 1u;     // observe only: no update, no push
constexpr uint32_t kWhatShift = 1u;   // 2 bits
constexpr uint32_t kAccum = 8u;       // decide (and store) the prior cell of the new state
constexpr uint32_t kExpLaw = 16u;     // w <- w exp(eps dt G), else w (1 + eps dt G)
constexpr uint32_t kFrozen = 32u;     // particles do not move

// Tags: per particle and binning, the bin the particle fell in (kNoBin when
// none), and its prior cell; rows of `stride` uint16 after the 7 value rows.
constexpr uint16_t kNoBin = 0xFFFF;

template <typename T, typename PT>
struct FinArgs {
    const PT* part;
    int32_t pcols, jpad, J, ncell, n_models;
    const int32_t* chunk_desc;    // 8 per chunk: model, col0, ncol, slot0, nslot, base (2 x 32 bits)
    const int32_t* model_slot;    // M + 1
    const int32_t* model_chunk;   // M + 1
    int32_t nchunk;
    int32_t parity;               // chi^2 shares go to chunk_chi[parity]
    double* chunk_chi;            // 2 (parity) * 2 * nchunk: chi2, chi2_inst shares
    const double* Y;
    const double* sigma;
    double* y;
    double* ys;
    double* delta;
    T* cvec;
    T* cellmean;
    double* cellmean64;
    const double* seg_stats;
    StatRow* ring;
    double g, mu;
    int32_t first, accum_cells;
    const int* flag;
    long long* d_step;            // [0] step counter, [1] statistics-block tickets
};

template <typename T>
struct ErangeArgs {
    const T* in;
    int64_t stride;
    const int32_t* tile_model;
    const int64_t* tile_p0;
    const int32_t* tile_cnt;
    const int32_t* block_tile0;
    const int32_t* block_slot0;
    const Pot<T>* pots;
    double* out;   // 2 * nslot
};

// Priors a step would use, per particle (readback).
template <typename T>
struct GatherArgs {
    const T* in;
    const uint16_t* tin;
    int64_t stride;
    const T* what;
    T* out;
    const int32_t* tile_model;
    const int64_t* tile_p0;
    const int32_t* tile_cnt;
    const int32_t* block_tile0;
    const Pot<T>* pots;
    const T* lctab;
    const float* lcetab;
    const T* erange;
    const T* flatw;
    const T* cellmean;
    Cells cells;
    const Exact* ex;              // FP64 constants and tables (device memory)
    int32_t what_mode;
    int32_t cellrow;
};

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
constexpr int kMlpTrainThreads = 64;   // samples per training block
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
    float* gpart;              // (batch / kMlpTrainThreads) x kMlpNP partial gradients
    float lr, beta1, beta2, adam_eps;
    double fallback;
    float* what;               // n priors
    const float* cellmean;     // histogram prior cell means
    int32_t cellrow;           // tag row of the prior cell
    int32_t nblk;              // blocks of the inference passes (<= kMlpMaxInferBlocks)
    double* red;               // nblk x 2 per-block partials
    double* stats;             // gmax, sum w, sum e, judge numerator, judge, fallback used, refreshes
    const int* flag;
};

// Prior cells of the state a.out (tags, and cell sums and counts into the cell
// columns of the partial slots) when the fused kernel observes without them.
hipError_t launch_cells(const StepArgs<float, float>& a, int pot_kind, int blocks, size_t lds, hipStream_t s);
hipError_t set_cells_lds_limit(size_t lds);

// One refresh of the learned prior: sample, nbatch Adam steps from step t0 + 1
// on, priors of every particle, judge and fallback.
hipError_t launch_mlp_refresh(const MlpArgs& a, int pot_kind, int t0, hipStream_t s);

template <typename T, typename PT>
hipError_t launch_step(const StepArgs<T, PT>& a, int pot_kind, uint64_t sig, int nbin, int ilp, int blocks,
                       int threads, size_t lds, hipStream_t s);
// One multipole step up to the observation of the new state: weight update,
// first kick and drift, the new coefficients, second kick.
template <typename T, typename PT>
hipError_t launch_mp_step(const StepArgs<T, PT>& a, const MpArgs<T>& mp, uint64_t sig, int nbin, int blocks,
                          const MpLds& lds, hipStream_t s);
// Coefficients of the particles in mp.src (and, with kick, the second kick).
template <typename T>
hipError_t launch_mp_build(const MpArgs<T>& mp, int blocks, const MpLds& lds, hipStream_t s, bool kick);
template <typename T, typename PT>
hipError_t set_mp_lds_limit(size_t lds);
template <typename T, typename PT>
hipError_t set_step_lds_limit(int pot_kind, size_t lds);
template <typename T, typename PT>
hipError_t launch_finalize(const FinArgs<T, PT>& a, hipStream_t s);
template <typename T>
hipError_t launch_erange(const ErangeArgs<T>& a, int pot_kind, int blocks, hipStream_t s);
template <typename T>
hipError_t launch_gather(const GatherArgs<T>& a, int pot_kind, int blocks, hipStream_t s);

}  // namespace m2m
