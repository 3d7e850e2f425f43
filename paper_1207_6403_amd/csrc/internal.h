// internal.h -- host-side context of the C ABI (not exported).
#pragma once
#include <string>
#include <vector>

#include "m2m.h"
#include "forms.h"

// Launch plan: tiles of threads * ilp particles (never straddling a model),
// contiguous tile ranges per block, one partial slot per (block, model) pair,
// and the column chunks of the finalise kernel.
struct Plan {
    int threads = 0, ilp = 0, bpc = 0;
    int64_t ntile = 0;
    int nblock = 0, nslot = 0;
    size_t lds = 0;
    int32_t* tile_model = nullptr;
    int64_t* tile_p0 = nullptr;
    int32_t* tile_cnt = nullptr;
    int32_t* block_tile0 = nullptr;
    int32_t* block_slot0 = nullptr;
    m2m::BlockDesc* block_desc = nullptr;
    int32_t* model_slot = nullptr;
    int32_t* chunk_desc = nullptr;   // 8 per finalise chunk: model, col0, ncol, slot0, nslot, base
    int64_t* slot_base = nullptr;    // per slot: index of its first column in `part`
    int32_t* slot_stride = nullptr;  // per slot: distance between its chunks
    void* part = nullptr;
    double* seg_stats = nullptr;
    double* erange_out = nullptr;
};

struct m2m_ctx {
    // configuration
    int prec = 0, update = 1, frozen = 0;
    double dt = 0, eps = 0, mu = 0, tau = 0;
    int M = 0, pot_kind = 0;
    std::vector<int64_t> off;
    std::vector<m2m_potential> pots;
    m2m_prior prior{};
    m2m_obs_layout lay{};
    std::vector<double> edges_host[M2M_MAX_BINNINGS];
    std::vector<double> gh_host[M2M_MAX_BINNINGS];   // Gauss-Hermite V_b then sigma_b (GH binnings)
    int ngh = 0;                                      // GH bins over all binnings
    std::vector<double> erange_host;
    std::vector<double> erange_user;   // the caller's (Emin, Emax) per model, if given
    std::vector<float> lce_host;   // per model: origin and inverse spacing of the uniform-E tables
    int64_t N = 0, stride = 0;
    int J = 0, JP = 0, NC = 0, pcols = 0, nedge = 0;
    alignas(16) unsigned char lay_bytes[sizeof(m2m::Layout<double>)] = {};
    uint64_t sig = 0;   // layout structure signature
    // self-consistent multipole (one model): its parameters, node radii, node
    // tables, interval sums, readback tables
    bool mp = false;
    m2m_potential mp_pot{};
    void* mp_tab = nullptr;
    void* mp_acc[2] = {nullptr, nullptr};   // accelerations of the state in state[k] (3 rows each)
    double* mp_rk = nullptr;
    double* mp_S = nullptr;
    double* mp_A64 = nullptr;
    double* mp_B64 = nullptr;
    // FP32 coefficient build: interval keys, counts and offsets, sorted copy, chunk partials
    uint16_t* mp_key = nullptr;
    uint32_t* mp_counts = nullptr;
    uint32_t* mp_offs = nullptr;
    uint32_t* mp_total = nullptr;
    float4* mp_sorted = nullptr;
    float* mp_part = nullptr;
    int mp_G = 0;
    int64_t mp_R = 0;
    int mp_maxchunk = 0;
    m2m::MpLds mp_lds{};
    // learned prior (FP32, one model): parameters and Adam moments, samples,
    // partial gradients, inference partials and statistics, Adam steps taken
    std::vector<float> mlp_init_host;
    float* mlp_theta = nullptr;
    float* mlp_m = nullptr;
    float* mlp_v = nullptr;
    float4* mlp_sub = nullptr;
    float* mlp_gpart = nullptr;
    double* mlp_red = nullptr;
    double* mlp_stats = nullptr;
    int mlp_nblk = 0;
    float* noalloc_scratch = nullptr;   // the device's static scratch (m2m_mlp_loss_grad_noalloc)
    std::string noalloc_error;          // why it is null, if it is
    int64_t mlp_t = 0;
    // prior cells accumulated by a kernel of their own (the fused kernel then
    // observes without them): its LDS bytes
    bool cells_apart = false;
    size_t cells_lds = 0;
    m2m::Cells cells{};
    // discrete tracers: CSR by bin (first, bin of each), per tracer V, 1/s,
    // 1/(sqrt(2 pi) s), update factors, smoothed sums, the likelihood's term of
    // G per particle, block partials; perm: CSR position of the caller's tracer k
    int trc_n = 0, trc_binning = -1, trc_nb = 0, trc_nblk = 0;
    double trc_lambda = 0;
    std::vector<int32_t> trc_perm;
    int32_t* trc_first = nullptr;
    int32_t* trc_tbin = nullptr;
    void *trc_V = nullptr, *trc_is = nullptr, *trc_nf = nullptr, *trc_cL = nullptr, *trc_cM = nullptr;
    void* trc_extra = nullptr;
    double *trc_part = nullptr, *trc_Ls = nullptr, *trc_Ms = nullptr, *trc_ll = nullptr;
    // device
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0, numCU = 0, max_lds = 0;
    void* state[2] = {nullptr, nullptr};
    void* what = nullptr;
    void* pots_d = nullptr;
    void* pots64 = nullptr;
    void* lctab = nullptr;
    void* lcetab = nullptr;
    void* rcetab = nullptr;
    void* exact_d = nullptr;
    double* lctab64 = nullptr;
    double* erange64 = nullptr;
    double* edges64 = nullptr;
    void* erange = nullptr;
    void* flatw = nullptr;
    void* cvec = nullptr;
    void* cellmean = nullptr;
    void* edges = nullptr;
    void* ghtab = nullptr;     // (V, 1/sigma) pairs, particle precision
    void* ghtab32 = nullptr;   // the same in FP32
    void* scratch_n = nullptr;
    double* shell_buf = nullptr;   // shell moments: block partials, edges, sums (allocated at first use)
    double *Y = nullptr, *sigma = nullptr, *y = nullptr, *ys = nullptr, *delta = nullptr;
    double* cellmean64 = nullptr;
    // finalise column chunks (launch-shape independent) and chi^2 shares
    int nchunk = 0;
    std::vector<int32_t> chunk_model_host, chunk_col0_host, chunk_ncol_host;
    int32_t* model_chunk = nullptr;
    std::vector<int32_t> model_chunk_host;
    double* chunk_chi = nullptr;
    m2m::StatRow* ring = nullptr;
    int* flag = nullptr;
    long long* bad_step = nullptr;
    long long* d_step = nullptr;
    Plan plan;
    std::vector<void*> allocs;
    // host state
    int64_t step = 0;
    m2m_status status = M2M_OK;
    std::string msg;
    m2m_launch launch{};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_k[2] = {0, 0};
    std::vector<hipEvent_t> events;
    double last_kernel_ms = 0;
    int64_t last_launches = 0;
};
