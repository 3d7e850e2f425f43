// runtime.h -- kernel argument blocks and launch helpers shared by the
// library's translation units (never exported through the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace m2m {

constexpr int kRing = 4096;          // statistics rows kept per model
// Per-lane trash slots after the fused kernel's LDS histograms and cell sums:
// scatters of particles outside every bin, or whose decision the FP64 fix-up
// takes later, land there instead of branching around the atomic.
constexpr int kTrash = 64;
// Open decisions (particle, mask) a wave of the FP32 fused kernel queues in LDS
// before re-taking them in FP64 (one chunk of ILP = 2).
constexpr int kFixQ = 128;
constexpr int kSlotsPerSplit = 32;   // partial slots in flight per finalise thread
constexpr int kFinCols = 32;         // columns per finalise block
constexpr int kFinGroups = 8;        // slot groups per column (256 threads)

// Where a block of the fused kernel starts, in one load: its tiles [t0, t1),
// its first partial slot, and its first segment (the run of tiles of one
// model): the model, the first particle, the particle count and the tile after
// the segment (later segments, rare, come from the tile tables).
struct BlockDesc {
    int32_t t0, t1, slot0, m0;
    int64_t p0;
    int32_t n0, tseg1;
};

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
    uint32_t state_bytes;   // bytes of a state buffer (value and tag rows)
    T* what;                // per-particle priors (stored modes)
    const int32_t* tile_model;
    const int64_t* tile_p0;
    const int32_t* tile_cnt;
    const int32_t* block_tile0;   // nblocks + 1
    const int32_t* block_slot0;   // first partial slot of each block
    const BlockDesc* block_desc;  // nblocks
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
    double* seg_stats;            // nslot * 4: (S, sum w, sum w^2, min w) per partial slot
    const T* edges;
    const double* edges64;        // the same edges in FP64
    const T* ghtab;               // Gauss-Hermite (V, 1/sigma) pairs (lay.ngh of them)
    const T* extra;               // kTracers: per particle, the tracer likelihood's term of G
    int32_t nedge;
    int32_t pcols, jpad;
    Layout<T> lay;
    Cells cells;
    const Exact* ex;              // FP64 constants and tables (device memory)
    T dt, eps, mu;
    uint32_t flags;               // kObserve | kWhat* | kAccum | kExpLaw | kFrozen | kTracers
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
constexpr uint32_t kTracers = 64u;    // G gains extra[p] (discrete tracers' likelihood)

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
    const Pot<double>* pots;      // FP64: E(0) of the particles as stored, in FP64
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

// e0, e1 (timing): events that take the step kernel's own start and end times.
template <typename T, typename PT>
hipError_t launch_step(const StepArgs<T, PT>& a, int pot_kind, uint64_t sig, int nbin, int ilp, int blocks,
                       int threads, size_t lds, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <typename T, typename PT>
hipError_t set_step_lds_limit(int pot_kind, size_t lds);
template <typename T, typename PT>
hipError_t launch_finalize(const FinArgs<T, PT>& a, hipStream_t s);
template <typename T>
hipError_t launch_erange(const ErangeArgs<T>& a, int pot_kind, int blocks, hipStream_t s);
template <typename T>
hipError_t launch_gather(const GatherArgs<T>& a, int pot_kind, int blocks, hipStream_t s);

}  // namespace m2m
