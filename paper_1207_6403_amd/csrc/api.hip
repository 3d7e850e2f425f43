// api.hip -- the C ABI (include/m2m.h): context, buffers, launch plan, HIP
// graphs, readbacks and the launch-shape autotuner.
//
// Device memory (HBM) layout of a context, N particles over all models:
//   state[2]  ping-pong particle buffers, 7 SoA rows of `stride` values
//             (x y z vx vy vz w) then nbin + 1 rows of `stride` uint16 tags
//             (the bin of each binning and the prior cell of the particle);
//             step n reads state[n & 1], writes the other, so a failed step
//             leaves the last good state untouched;
//   what      per-particle priors (periodic and learned priors only);
//   per model observables y, ys, delta (FP64, J each), the FP32/FP64 update
//             table Dt_j/sigma_j, prior cell means, chi^2, a statistics ring;
//   partial   one slot per (block, model) pair: the block's LDS histograms,
//             summed in fixed order by the finalise kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "m2m.h"
#include "runtime.h"
#include "internal.h"

using namespace m2m;

static thread_local std::string g_create_error;

// ------------------------------------------------------------------ helpers
namespace {

m2m_status fail(m2m_ctx* c, m2m_status s, const std::string& msg) {
    if (c) { c->msg = msg; }
    else g_create_error = msg;
    return s;
}

#define HIPCHK(ctx, expr)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, M2M_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_));    \
    } while (0)

template <typename X>
m2m_status dalloc(m2m_ctx* c, X** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(X));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(c, M2M_ERR_NOMEM, "hipMalloc of " + std::to_string(n * sizeof(X)) + " bytes failed");
    }
    c->allocs.push_back((void*)*p);
    return M2M_OK;
}

void dfree(m2m_ctx* c, void* p) {
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
    (void)hipFree(p);
}

size_t tsize(const m2m_ctx* c) { return c->prec == M2M_F64 ? 8 : 4; }

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

// --------------------------------------------------------------- validation
static m2m_status check_potential(const m2m_potential& p) {
    if (p.kind == M2M_POT_HERNQUIST || p.kind == M2M_POT_HERNQUIST_NFW) {
        if (!(p.G > 0 && p.M >= 0 && p.a > 0)) return fail(nullptr, M2M_ERR_INVALID, "Hernquist needs G>0, M>=0, a>0");
        if (p.kind == M2M_POT_HERNQUIST_NFW && !(p.Mh >= 0 && p.rs > 0))
            return fail(nullptr, M2M_ERR_INVALID, "NFW needs Mh>=0, rs>0");
    } else if (p.kind == M2M_POT_LOG) {
        if (!(p.v0 > 0 && p.Rc > 0 && p.q > 0)) return fail(nullptr, M2M_ERR_INVALID, "log potential needs v0, Rc, q > 0");
    } else if (p.kind == M2M_POT_MULTIPOLE) {
        if (!(p.lmax >= 0 && p.lmax <= 8 && p.nnode >= 2 && p.nnode <= 512 && p.rmin > 0 && p.rmax > p.rmin &&
              p.G > 0 && p.Mtot > 0))
            return fail(nullptr, M2M_ERR_INVALID, "multipole needs 0<=lmax<=8, 2<=nnode<=512, 0<rmin<rmax, G, Mtot > 0");
    } else {
        return fail(nullptr, M2M_ERR_INVALID, "unknown potential kind");
    }
    return M2M_OK;
}

static m2m_status validate(const m2m_config* cfg, const m2m_obs_layout* lay, const m2m_target* tg,
                           int64_t* N_out, int* J_out) {
    if (!cfg || !lay || !tg) return fail(nullptr, M2M_ERR_INVALID, "null config, layout or target");
    if (cfg->abi_version != M2M_ABI_VERSION) return fail(nullptr, M2M_ERR_INVALID, "abi_version mismatch");
    if (cfg->precision != M2M_F32 && cfg->precision != M2M_F64) return fail(nullptr, M2M_ERR_INVALID, "precision");
    if (cfg->update != M2M_UPDATE_EULER && cfg->update != M2M_UPDATE_EXP) return fail(nullptr, M2M_ERR_INVALID, "update");
    if (!(cfg->dt > 0) || !is_fin(cfg->dt)) return fail(nullptr, M2M_ERR_INVALID, "dt must be > 0");
    if (!(cfg->eps >= 0) || !is_fin(cfg->eps)) return fail(nullptr, M2M_ERR_INVALID, "eps must be >= 0");
    if (!(cfg->mu >= 0) || !is_fin(cfg->mu)) return fail(nullptr, M2M_ERR_INVALID, "mu must be >= 0");
    if (!(cfg->tau >= cfg->dt) || !is_fin(cfg->tau)) return fail(nullptr, M2M_ERR_INVALID, "tau must be >= dt");
    if (cfg->n_models < 1 || !cfg->model_offsets || !cfg->potentials)
        return fail(nullptr, M2M_ERR_INVALID, "n_models >= 1 with offsets and potentials required");
    if (cfg->model_offsets[0] != 0) return fail(nullptr, M2M_ERR_INVALID, "model_offsets[0] must be 0");
    for (int m = 0; m < cfg->n_models; ++m)
        if (cfg->model_offsets[m + 1] <= cfg->model_offsets[m])
            return fail(nullptr, M2M_ERR_INVALID, "every model needs at least one particle (offsets increasing)");
    const int kind = cfg->potentials[0].kind;
    for (int m = 0; m < cfg->n_models; ++m) {
        const m2m_potential& p = cfg->potentials[m];
        if (p.kind != kind) return fail(nullptr, M2M_ERR_INVALID, "all models must share the potential kind");
        const m2m_status ps = check_potential(p);
        if (ps) return ps;
    }
    if (lay->nbin < 1 || lay->nbin > M2M_MAX_BINNINGS) return fail(nullptr, M2M_ERR_INVALID, "nbin must be 1..4");
    if (!is_fin(lay->incl)) return fail(nullptr, M2M_ERR_INVALID, "inclination");
    int J = 0, ne = 0;
    for (int b = 0; b < lay->nbin; ++b) {
        const m2m_binning& d = lay->bin[b];
        if (d.nmom < 1 || d.nmom > 3) return fail(nullptr, M2M_ERR_INVALID, "nmom must be 1..3");
        bool gh = false;
        for (int k = 0; k < d.nmom; ++k) {
            if (d.mom[k] < M2M_MOM_MASS || d.mom[k] > M2M_MOM_H4)
                return fail(nullptr, M2M_ERR_INVALID, "moment codes are 0..6");
            gh |= d.mom[k] >= M2M_MOM_H1;
        }
        int nb;
        if (d.kind == M2M_BIN_SHELL || d.kind == M2M_BIN_ANNULUS) {
            if (d.nedge < 2 || !d.edges) return fail(nullptr, M2M_ERR_INVALID, "need >= 2 edges");
            for (int k = 0; k < d.nedge; ++k) {
                if (!is_fin(d.edges[k])) return fail(nullptr, M2M_ERR_INVALID, "edges must be finite");
                if (k && !(d.edges[k] > d.edges[k - 1])) return fail(nullptr, M2M_ERR_INVALID, "edges must increase");
            }
            nb = d.nedge - 1;
            ne += d.nedge;
        } else if (d.kind == M2M_BIN_GRID) {
            if (d.nx < 1 || d.ny < 1 || !(d.x1 > d.x0) || !(d.y1 > d.y0) || !is_fin(d.x0) || !is_fin(d.x1) ||
                !is_fin(d.y0) || !is_fin(d.y1))
                return fail(nullptr, M2M_ERR_INVALID, "grid needs nx, ny >= 1 and x1 > x0, y1 > y0");
            nb = d.nx * d.ny;
        } else {
            return fail(nullptr, M2M_ERR_INVALID, "unknown binning kind");
        }
        if (nb > 65534) return fail(nullptr, M2M_ERR_UNSUPPORTED, "at most 65534 bins per binning");
        if (gh) {
            if (!d.gh) return fail(nullptr, M2M_ERR_INVALID, "Gauss-Hermite moments need the bins' (V, sigma)");
            for (int k = 0; k < nb; ++k)
                if (!is_fin(d.gh[k]) || !(d.gh[nb + k] > 0) || !is_fin(d.gh[nb + k]))
                    return fail(nullptr, M2M_ERR_INVALID, "Gauss-Hermite V must be finite and sigma > 0");
        }
        J += d.nmom * nb;
    }
    if (ne > M2M_MAX_EDGES) return fail(nullptr, M2M_ERR_INVALID, "too many edges (max 256)");
    if (tg->J != J) return fail(nullptr, M2M_ERR_INVALID, "target J does not match the layout");
    if (!tg->Y || !tg->sigma) return fail(nullptr, M2M_ERR_INVALID, "target arrays missing");
    const int64_t nt = (int64_t)J * (tg->per_model ? cfg->n_models : 1);
    for (int64_t j = 0; j < nt; ++j)
        if (!is_fin(tg->Y[j]) || !(tg->sigma[j] > 0) || !is_fin(tg->sigma[j]))
            return fail(nullptr, M2M_ERR_INVALID, "target Y must be finite and sigma > 0");
    const m2m_prior& P = cfg->prior;
    if (P.kind != M2M_PRIOR_FLAT && P.kind != M2M_PRIOR_HIST && P.kind != M2M_PRIOR_MLP)
        return fail(nullptr, M2M_ERR_INVALID, "unknown prior kind");
    if (P.kind != M2M_PRIOR_FLAT) {
        if (P.n[0] < 1 || P.n[1] < 1 || P.n[2] < 1 || (int64_t)P.n[0] * P.n[1] * P.n[2] > 16384)
            return fail(nullptr, M2M_ERR_INVALID, "prior cells must be >= 1 per axis, <= 16384 in all");
        if (P.ax2 != 0 && P.ax2 != 1) return fail(nullptr, M2M_ERR_INVALID, "prior ax2 must be 0 or 1");
        if (P.period < 1) return fail(nullptr, M2M_ERR_INVALID, "prior period must be >= 1");
        if (P.Erange)
            for (int m = 0; m < cfg->n_models; ++m)
                if (!(P.Erange[2 * m + 1] > P.Erange[2 * m]) || !is_fin(P.Erange[2 * m]) || !is_fin(P.Erange[2 * m + 1]))
                    return fail(nullptr, M2M_ERR_INVALID, "prior Erange needs Emin < Emax per model");
        if (kind == M2M_POT_MULTIPOLE) {
            if (P.ref.kind < 0 || P.ref.kind == M2M_POT_MULTIPOLE)
                return fail(nullptr, M2M_ERR_INVALID, "multipole models need an analytic prior reference potential");
            const m2m_status rs = check_potential(P.ref);
            if (rs) return rs;
        } else if (P.ref.kind >= 0 && P.ref.kind != kind) {
            return fail(nullptr, M2M_ERR_UNSUPPORTED, "prior reference potential must be the model potential here");
        }
    }
    if (P.kind == M2M_PRIOR_MLP) {
        if (!P.mlp_init) return fail(nullptr, M2M_ERR_INVALID, "learned prior needs mlp_init");
        if (P.mlp_batch < kMlpSamples || P.mlp_batch % kMlpSamples || P.mlp_subset < P.mlp_batch ||
            P.mlp_subset % P.mlp_batch)
            return fail(nullptr, M2M_ERR_INVALID, "mlp_batch must be a multiple of 32 and divide mlp_subset");
        if (!(P.lr > 0) || !(P.beta1 >= 0 && P.beta1 < 1) || !(P.beta2 >= 0 && P.beta2 < 1) || !(P.adam_eps >= 0) ||
            !(P.fallback >= 0))
            return fail(nullptr, M2M_ERR_INVALID, "learned prior needs lr > 0, 0 <= beta < 1, adam_eps >= 0, fallback >= 0");
        for (int k = 0; k < M2M_MLP_NPARAM; ++k)
            if (!is_fin(P.mlp_init[k])) return fail(nullptr, M2M_ERR_INVALID, "mlp_init must be finite");
        if (cfg->n_models != 1) return fail(nullptr, M2M_ERR_UNSUPPORTED, "the learned prior runs on one model per context");
        if (cfg->precision != M2M_F32) return fail(nullptr, M2M_ERR_UNSUPPORTED, "the learned prior runs in FP32 contexts");
        if (cfg->model_offsets[1] >= ((int64_t)1 << 32))
            return fail(nullptr, M2M_ERR_UNSUPPORTED, "the learned prior samples at most 2^32 particles");
    }
    if (kind == M2M_POT_MULTIPOLE && cfg->n_models != 1)
        return fail(nullptr, M2M_ERR_UNSUPPORTED, "a multipole model runs alone in its context");
    *N_out = cfg->model_offsets[cfg->n_models];
    *J_out = J;
    return M2M_OK;
}

// ------------------------------------------------------------------ the plan
static void free_plan(m2m_ctx* c) {
    Plan& p = c->plan;
    for (void* q : {(void*)p.tile_model, (void*)p.tile_p0, (void*)p.tile_cnt, (void*)p.block_tile0,
                    (void*)p.block_slot0, (void*)p.block_desc, (void*)p.model_slot, (void*)p.part, (void*)p.seg_stats,
                    (void*)p.erange_out, (void*)p.chunk_desc, (void*)p.slot_base, (void*)p.slot_stride})
        dfree(c, q);
    p = Plan();
    for (int k = 0; k < 2; ++k)
        if (c->graph[k]) { (void)hipGraphExecDestroy(c->graph[k]); c->graph[k] = nullptr; }
}

template <typename X>
static m2m_status upload(m2m_ctx* c, X** d, const std::vector<X>& h) {
    m2m_status s = dalloc(c, d, h.size());
    if (s) return s;
    HIPCHK(c, hipMemcpy(*d, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice));
    return M2M_OK;
}

static m2m_status make_plan(m2m_ctx* c, int threads, int ilp, int bpc) {
    free_plan(c);
    Plan& p = c->plan;
    p.threads = threads;
    p.ilp = ilp;
    p.bpc = bpc;
    const int64_t TS = (int64_t)threads * ilp;
    std::vector<int32_t> tm, tc;
    std::vector<int64_t> tp;
    for (int m = 0; m < c->M; ++m) {
        const int64_t n = c->off[m + 1] - c->off[m];
        for (int64_t k = 0; k * TS < n; ++k) {
            tm.push_back(m);
            tp.push_back(c->off[m] + k * TS);
            tc.push_back((int32_t)std::min<int64_t>(TS, n - k * TS));
        }
    }
    const int64_t T = (int64_t)tm.size();
    const int64_t B = std::max<int64_t>(1, std::min<int64_t>(T, (int64_t)c->numCU * bpc));
    std::vector<int32_t> bt0(B + 1), bs0(B), mslot(c->M + 1, -1);
    int32_t nslot = 0;
    for (int64_t b = 0; b <= B; ++b) bt0[b] = (int32_t)((b * T) / B);
    for (int64_t b = 0; b < B; ++b) {
        bs0[b] = nslot;
        if (bt0[b] == bt0[b + 1]) continue;
        const int mlo = tm[bt0[b]], mhi = tm[bt0[b + 1] - 1];
        for (int m = mlo; m <= mhi; ++m) {
            if (mslot[m] < 0) mslot[m] = nslot;
            ++nslot;
        }
    }
    mslot[c->M] = nslot;
    std::vector<BlockDesc> bdesc(B);
    for (int64_t b = 0; b < B; ++b) {
        BlockDesc& d = bdesc[b];
        d = BlockDesc{};
        d.t0 = bt0[b];
        d.t1 = bt0[b + 1];
        d.slot0 = bs0[b];
        if (d.t0 < d.t1) {
            d.m0 = tm[d.t0];
            d.p0 = tp[d.t0];
            int32_t te = d.t0;
            while (te < d.t1 && tm[te] == d.m0) ++te;
            d.n0 = (int32_t)(tp[te - 1] + tc[te - 1] - tp[d.t0]);
            d.tseg1 = te;
        } else {
            d.tseg1 = d.t1;
        }
    }
    p.ntile = T;
    p.nblock = (int)B;
    p.nslot = nslot;
    m2m_status s;
    if ((s = upload(c, &p.tile_model, tm)) || (s = upload(c, &p.tile_p0, tp)) || (s = upload(c, &p.tile_cnt, tc)) ||
        (s = upload(c, &p.block_tile0, bt0)) || (s = upload(c, &p.block_slot0, bs0)) ||
        (s = upload(c, &p.block_desc, bdesc)) || (s = upload(c, &p.model_slot, mslot)))
        return s;
    // partial slots, chunk-major: for model m, chunk k (kFinCols columns) of all
    // the model's slots is one contiguous block, so each finalise block reads
    // one contiguous range
    const int cpm = c->nchunk / c->M;   // chunks per model
    std::vector<int64_t> mbase(c->M + 1, 0), sbase(nslot);
    std::vector<int32_t> sstride(nslot);
    for (int m = 0; m < c->M; ++m) {
        const int ns = mslot[m + 1] - mslot[m];
        mbase[m + 1] = mbase[m] + (int64_t)cpm * ns * kFinCols;
        for (int q = mslot[m]; q < mslot[m + 1]; ++q) {
            sbase[q] = mbase[m] + (int64_t)(q - mslot[m]) * kFinCols;
            sstride[q] = ns * kFinCols;
        }
    }
    // finalise chunk descriptors: model, first column, columns, first slot,
    // slots, start of the chunk's block of partials (low, high 32 bits)
    std::vector<int32_t> desc(8 * (size_t)c->nchunk, 0);
    for (int k = 0; k < c->nchunk; ++k) {
        const int m = c->chunk_model_host[k];
        const int ns = mslot[m + 1] - mslot[m];
        const int64_t base = mbase[m] + (int64_t)(c->chunk_col0_host[k] / kFinCols) * ns * kFinCols;
        desc[8 * k] = m;
        desc[8 * k + 1] = c->chunk_col0_host[k];
        desc[8 * k + 2] = c->chunk_ncol_host[k];
        desc[8 * k + 3] = mslot[m];
        desc[8 * k + 4] = ns;
        desc[8 * k + 5] = (int32_t)(base & 0xffffffff);
        desc[8 * k + 6] = (int32_t)(base >> 32);
    }
    const size_t npart = (size_t)mbase[c->M];
    if ((s = upload(c, &p.chunk_desc, desc)) || (s = upload(c, &p.slot_base, sbase)) ||
        (s = upload(c, &p.slot_stride, sstride)))
        return s;
    // per-wave statistics rows, the identity where no wave writes
    std::vector<double> st0((size_t)nslot * 4, 0.0);
    for (size_t r = 0; r < (size_t)nslot; ++r) st0[4 * r + 3] = INFINITY;
    if ((s = dalloc(c, (char**)&p.part, npart * tsize(c))) || (s = upload(c, &p.seg_stats, st0)) ||
        (s = dalloc(c, &p.erange_out, (size_t)nslot * 2)))
        return s;
    HIPCHK(c, hipMemset(p.part, 0, npart * tsize(c)));
    // LDS of the fused kernel: histograms, cell sums/counts, update table,
    // cell means, edges, reduction scratch, Lc table
    const size_t ts = tsize(c);
    const int NCk = c->cells_apart ? 0 : c->NC;   // cells the fused kernel holds
    const int NCe = (NCk + 1) & ~1, NE = (c->nedge + 1) & ~1;
    p.lds = 8 * ((size_t)c->JP + kTrash + NCk + kTrash + NE + 2 + 64) + 4 * ((size_t)NCe + kTrash) +
            ts * ((size_t)c->JP + 2 + NCe + NE + kLcTab) + (ts == 4 && NCk > 0 ? 8 * (size_t)kLcE : 0) +
            (ts == 4 ? 8 * (size_t)kFixQ * (threads / 64) : 0) + ts * 2 * (size_t)c->ngh;
    p.lds = (p.lds + 15) & ~(size_t)15;
    if (p.lds > (size_t)c->max_lds)
        return fail(c, M2M_ERR_UNSUPPORTED, "layout needs " + std::to_string(p.lds) + " bytes of LDS per block (max " +
                                                std::to_string(c->max_lds) + ")");
    if (c->mp) {
        // multipole kernels: the FP32 second kick keeps the node table in LDS (the
        // first kick reads the stored field and needs no table)
        const int nn = c->mp_pot.nnode;
        const bool f32 = ts == 4;
        MpLds& L = c->mp_lds;
        L.kick_drift = 512;
        L.coeff = 0;
        L.kick = f32 ? 4 * (size_t)nn * kMpRowF : 0;
        const size_t need = std::max(L.kick_drift, L.kick);
        if (need > (size_t)c->max_lds)
            return fail(c, M2M_ERR_UNSUPPORTED, "multipole with " + std::to_string(nn) + " nodes needs " +
                                                    std::to_string(need) + " bytes of LDS per block (max " +
                                                    std::to_string(c->max_lds) + ")");
    }
    return M2M_OK;
}

// --------------------------------------------------------------- launches
static const Exact* exact_tables(const m2m_ctx* c) { return (const Exact*)c->exact_d; }

template <typename T>
static Layout<T> layout_of(const m2m_ctx* c);

// FP64 constants and table pointers of the exact decisions, uploaded once.
static m2m_status upload_exact(m2m_ctx* c) {
    Exact e{};
    e.pots = (const Pot<double>*)c->pots64;
    e.lctab = c->lctab64;
    e.erange = c->erange64;
    e.edges = c->edges64;
    e.rce = (const float*)c->rcetab;
    e.gh = (const float*)c->ghtab32;
    e.lay = layout_of<float>(c);
    e.cells = c->cells;
    e.cosd = std::cos(c->lay.incl);
    e.sind = std::sin(c->lay.incl);
    for (int b = 0; b < c->lay.nbin; ++b) {
        const m2m_binning& d = c->lay.bin[b];
        if (d.kind != M2M_BIN_GRID) continue;
        e.x0d[b] = d.x0;
        e.wxd[b] = d.x1 - d.x0;
        e.y0d[b] = d.y0;
        e.wyd[b] = d.y1 - d.y0;
    }
    std::vector<unsigned char> h(sizeof(Exact));
    std::memcpy(h.data(), &e, sizeof(e));
    return upload(c, (unsigned char**)&c->exact_d, h);
}

// Tag rows of state buffer k.
static uint16_t* tags(const m2m_ctx* c, int k) {
    return (uint16_t*)((char*)c->state[k] + (size_t)7 * c->stride * tsize(c));
}

static size_t state_bytes(const m2m_ctx* c);

template <typename T>
static void fill_step_args(m2m_ctx* c, StepArgs<T, T>& a, int parity, int mode, int what_mode, int accum) {
    const Plan& p = c->plan;
    a.in = (const T*)c->state[parity];
    a.out = (T*)c->state[parity ^ 1];
    a.stride = c->stride;
    a.state_bytes = (uint32_t)state_bytes(c);
    a.what = (T*)c->what;
    a.tile_model = p.tile_model;
    a.tile_p0 = p.tile_p0;
    a.tile_cnt = p.tile_cnt;
    a.block_tile0 = p.block_tile0;
    a.block_slot0 = p.block_slot0;
    a.block_desc = p.block_desc;
    a.pots = (const Pot<T>*)c->pots_d;
    a.lctab = (const T*)c->lctab;
    a.lcetab = (const float*)c->lcetab;
    a.erange = (const T*)c->erange;
    a.flatw = (const T*)c->flatw;
    a.cvec = (const T*)c->cvec;
    a.cellmean = (const T*)c->cellmean;
    a.part = (T*)p.part;
    a.slot_base = p.slot_base;
    a.slot_stride = p.slot_stride;
    a.seg_stats = p.seg_stats;
    a.edges = (const T*)c->edges;
    a.edges64 = c->edges64;
    a.ghtab = (const T*)c->ghtab;
    a.extra = nullptr;
    a.nedge = c->nedge;
    a.pcols = c->pcols;
    a.jpad = c->JP;
    std::memcpy(&a.lay, c->lay_bytes, sizeof(Layout<T>));
    a.cells = c->cells;
    a.ex = exact_tables(c);
    a.dt = (T)c->dt;
    a.eps = (T)c->eps;
    a.mu = (T)c->mu;
    if (c->cells_apart) {
        // the cells are accumulated by their own kernel (launch_cells_after)
        a.cells.ncell = 0;
        accum = 0;
    }
    // (an observe-only pass neither updates nor moves: the law and frozen flags
    // are left out, so that it matches the compiled-in observe flags)
    a.flags = mode == 1 ? kObserve | ((uint32_t)what_mode << kWhatShift) | (accum ? kAccum : 0u)
                        : ((uint32_t)what_mode << kWhatShift) | (accum ? kAccum : 0u) |
                              (c->update == 1 ? kExpLaw : 0u) | (c->frozen ? kFrozen : 0u);
    a.cellrow = c->lay.nbin;
    a.flag = c->flag;
    a.bad_step = c->bad_step;
    a.d_step = c->d_step;
}

template <typename T>
static void fill_fin_args(m2m_ctx* c, FinArgs<T, T>& f, int first, int accum, int parity) {
    const Plan& p = c->plan;
    f.part = (const T*)p.part;
    f.pcols = c->pcols;
    f.jpad = c->JP;
    f.J = c->J;
    f.ncell = c->NC;
    f.n_models = c->M;
    f.chunk_desc = p.chunk_desc;
    f.model_slot = p.model_slot;
    f.model_chunk = c->model_chunk;
    f.nchunk = c->nchunk;
    f.parity = parity;
    f.chunk_chi = c->chunk_chi;
    f.Y = c->Y;
    f.sigma = c->sigma;
    f.y = c->y;
    f.ys = c->ys;
    f.delta = c->delta;
    f.cvec = (T*)c->cvec;
    f.cellmean = (T*)c->cellmean;
    f.cellmean64 = c->cellmean64;
    f.seg_stats = p.seg_stats;
    f.ring = c->ring;
    f.g = c->dt / c->tau;
    f.mu = c->mu;
    f.first = first;
    f.accum_cells = accum;
    f.flag = c->flag;
    f.d_step = c->d_step;
}

// prior handling of step n: (what_mode, accumulate cells for step n+1)
static void prior_modes(const m2m_ctx* c, int64_t n, int* what_mode, int* accum) {
    const int P = c->prior.period;
    if (c->prior.kind == M2M_PRIOR_FLAT) { *what_mode = 0; *accum = 0; }
    else if (c->prior.kind == M2M_PRIOR_HIST && P == 1) { *what_mode = 1; *accum = 1; }
    else if (c->prior.kind == M2M_PRIOR_HIST) { *what_mode = (n % P == 0) ? 2 : 3; *accum = ((n + 1) % P == 0); }
    else { *what_mode = 3; *accum = ((n + 1) % P == 0); }   // learned: refreshed before step n when n % P == 0
}

// Multipole kernel arguments; src is the state buffer the coefficient and
// second-kick kernels work on.
template <typename T>
static void fill_mp_args(const m2m_ctx* c, MpArgs<T>& mp, const void* src, int parity, int kick) {
    const m2m_potential& q = c->mp_pot;
    const Plan& p = c->plan;
    const double lr0 = std::log(q.rmin), dl = (std::log(q.rmax) - lr0) / (q.nnode - 1);
    mp.lmax = q.lmax;
    mp.nn = q.nnode;
    mp.nlm = (q.lmax + 1) * (q.lmax + 1);
    mp.nblock = p.nblock;
    mp.lr0 = (T)lr0;
    mp.idl = (T)(1.0 / dl);
    mp.rmin = (T)q.rmin;
    mp.rmax = (T)q.rmax;
    mp.G = (T)q.G;
    mp.Mtot = (T)q.Mtot;
    mp.hdt = (T)(0.5 * c->dt);
    mp.lr0d = lr0;
    mp.dld = dl;
    mp.tab = (const T*)c->mp_tab;
    mp.tab_out = (T*)c->mp_tab;
    mp.rk = c->mp_rk;
    mp.n = c->N;
    mp.G_sort = c->mp_G;
    mp.R = c->mp_R;
    mp.maxchunk = c->mp_maxchunk;
    mp.key = c->mp_key;
    mp.counts = c->mp_counts;
    mp.offs = c->mp_offs;
    mp.total = c->mp_total;
    mp.sorted = c->mp_sorted;
    mp.part = c->mp_part;
    mp.S = c->mp_S;
    mp.A64 = c->mp_A64;
    mp.B64 = c->mp_B64;
    mp.src = (const T*)src;
    mp.stride = c->stride;
    mp.acc_in = (const T*)c->mp_acc[parity];
    mp.acc_out = (T*)c->mp_acc[parity ^ 1];
    mp.kick = kick;
    mp.block_tile0 = p.block_tile0;
    mp.tile_p0 = p.tile_p0;
    mp.tile_cnt = p.tile_cnt;
    mp.flag = c->flag;
}

// When the cells are kept apart: the cells of the state in buffer k, after the
// fused kernel has observed it.
template <typename T>
static hipError_t launch_cells_after(m2m_ctx* c, int k) {
    if constexpr (sizeof(T) == 4) {
        StepArgs<float, float> a;
        fill_step_args<float>(c, a, k ^ 1, 1, 0, 1);
        a.out = (float*)c->state[k];
        a.cells = c->cells;
        return launch_cells(a, c->pot_kind, c->plan.nblock, c->cells_lds, c->stream);
    }
    return hipSuccess;
}

// Learned-prior kernel arguments for the refresh before step n (state n).
static void fill_mlp_args(const m2m_ctx* c, MlpArgs& a, int64_t n) {
    const m2m_prior& P = c->prior;
    a.state = (const float*)c->state[n & 1];
    a.stride = c->stride;
    a.n = c->N;
    a.ex = exact_tables(c);
    a.lcE0 = c->lce_host[0];
    a.lcEinv = c->lce_host[1];
    a.Emin = c->erange_host[0];
    a.Emax = c->erange_host[1];
    a.seed = P.seed;
    a.q = (uint32_t)(n / P.period);
    a.subset = P.mlp_subset;
    a.batch = P.mlp_batch;
    a.sub = c->mlp_sub;
    a.theta = c->mlp_theta;
    a.adam_m = c->mlp_m;
    a.adam_v = c->mlp_v;
    a.gpart = c->mlp_gpart;
    a.lr = (float)P.lr;
    a.beta1 = (float)P.beta1;
    a.beta2 = (float)P.beta2;
    a.adam_eps = (float)P.adam_eps;
    a.fallback = P.fallback;
    a.what = (float*)c->what;
    a.cellmean = (const float*)c->cellmean;
    a.cellrow = c->lay.nbin;
    a.nblk = c->mlp_nblk;
    a.red = c->mlp_red;
    a.stats = c->mlp_stats;
    a.loss = nullptr;
    a.mfma = P.mlp_mfma;
    a.pot32 = P.mlp_mfma && !c->mp ? (const Pot<float>*)c->pots_d : nullptr;
    a.lcetab = (const float2*)c->lcetab;
    a.flag = c->flag;
}

// Priors what_i of the particles in state buffer k from their cell tags and the
// cell means (or per particle, flat or held), into out.
template <typename T>
static GatherArgs<T> gather_args(m2m_ctx* c, int k, int what_mode, T* out) {
    GatherArgs<T> a;
    a.in = (const T*)c->state[k];
    a.tin = tags(c, k);
    a.stride = c->stride;
    a.what = (const T*)c->what;
    a.out = out;
    a.tile_model = c->plan.tile_model;
    a.tile_p0 = c->plan.tile_p0;
    a.tile_cnt = c->plan.tile_cnt;
    a.block_tile0 = c->plan.block_tile0;
    a.pots = (const Pot<T>*)c->pots_d;
    a.lctab = (const T*)c->lctab;
    a.lcetab = (const float*)c->lcetab;
    a.erange = (const T*)c->erange;
    a.flatw = (const T*)c->flatw;
    a.cellmean = (const T*)c->cellmean;
    a.cells = c->cells;
    a.ex = exact_tables(c);
    a.what_mode = what_mode;
    a.cellrow = c->lay.nbin;
    return a;
}

// Tracer kernels' arguments for the state in buffer k.
template <typename T>
static TracerArgs<T> tracer_args(const m2m_ctx* c, int k, int first_obs) {
    TracerArgs<T> a{};
    a.state = (const T*)c->state[k];
    a.stride = c->stride;
    a.n = c->N;
    a.tagrow = c->trc_binning;
    a.ntr = c->trc_n;
    a.nb = c->trc_nb;
    a.sini = (T)std::sin(c->lay.incl);
    a.cosi = (T)std::cos(c->lay.incl);
    a.first = c->trc_first;
    a.V = (const T*)c->trc_V;
    a.is = (const T*)c->trc_is;
    a.nf = (const T*)c->trc_nf;
    a.cL = (const T*)c->trc_cL;
    a.cM = (const T*)c->trc_cM;
    a.extra = (T*)c->trc_extra;
    a.part = c->trc_part;
    a.nblk = c->trc_nblk;
    a.Ls = c->trc_Ls;
    a.Ms = c->trc_Ms;
    a.cL_out = (T*)c->trc_cL;
    a.cM_out = (T*)c->trc_cM;
    a.loglike = c->trc_ll;
    a.tbin = c->trc_tbin;
    a.g = c->dt / c->tau;
    a.lambda = c->trc_lambda;
    a.first_obs = first_obs;
    a.flag = c->flag;
    return a;
}

template <typename T>
static hipError_t launch_one_T(m2m_ctx* c, int64_t n, hipEvent_t e0, hipEvent_t e1) {
    int wm, acc;
    prior_modes(c, n, &wm, &acc);
    if (c->cells_apart && (wm == 1 || wm == 2)) {
        // the fused kernel holds no cell means: gather the priors first and step
        // with them as held priors
        const hipError_t e = launch_gather<T>(gather_args<T>(c, (int)(n & 1), 1, (T*)c->what), c->pot_kind,
                                              c->plan.nblock, c->stream);
        if (e != hipSuccess) return e;
        wm = 3;
    }
    StepArgs<T, T> a;
    fill_step_args<T>(c, a, (int)(n & 1), 0, wm, acc);
    const Plan& p = c->plan;
    if constexpr (sizeof(T) == 4) {
        if (c->prior.kind == M2M_PRIOR_MLP && n % c->prior.period == 0) {
            // learned prior: refresh on state n before its update
            MlpArgs m;
            fill_mlp_args(c, m, n);
            const hipError_t e = launch_mlp_refresh(m, c->pot_kind, (int)c->mlp_t, c->stream);
            if (e != hipSuccess) return e;
            c->mlp_t += c->prior.mlp_subset / c->prior.mlp_batch;
        }
    }
    hipError_t e;
    if (c->mp) {
        // self-consistent model: update, kicks and drift with the coefficient
        // rebuild between them, then the fused kernel observes the new state
        // (the timing events bracket the second kick, which evaluates the field)
        MpArgs<T> mp;
        fill_mp_args<T>(c, mp, a.out, (int)(n & 1), 1);
        e = launch_mp_step<T, T>(a, mp, c->sig, c->lay.nbin, p.nblock, c->mp_lds, c->stream);
        if (e == hipSuccess && !c->frozen) e = launch_mp_build<T>(mp, p.nblock, c->mp_lds, c->stream, e0, e1);
        e0 = e1 = nullptr;
        if (e == hipSuccess) {
            StepArgs<T, T> o;
            fill_step_args<T>(c, o, (int)((n + 1) & 1), 1, 0, acc);
            o.out = (T*)c->state[(n + 1) & 1];
            e = launch_step<T, T>(o, c->pot_kind, c->sig, c->lay.nbin, p.ilp, p.nblock, p.threads, p.lds, c->stream);
        }
    } else {
        if (c->trc_n) {
            // the tracers' term of G for every particle of state n
            if ((e = launch_tracer_grad<T>(tracer_args<T>(c, (int)(n & 1), 0), c->stream)) != hipSuccess) return e;
            a.flags |= kTracers;
            a.extra = (const T*)c->trc_extra;
        }
        // (timing: the events take the step kernel's own start and end times)
        e = launch_step<T, T>(a, c->pot_kind, c->sig, c->lay.nbin, p.ilp, p.nblock, p.threads, p.lds, c->stream, e0,
                              e1);
    }
    if (e != hipSuccess) return e;
    if (c->cells_apart && acc && (e = launch_cells_after<T>(c, (int)((n + 1) & 1))) != hipSuccess) return e;
    if (c->trc_n && (e = launch_tracer_observe<T>(tracer_args<T>(c, (int)((n + 1) & 1), 0), c->stream)) != hipSuccess)
        return e;
    FinArgs<T, T> f;
    fill_fin_args<T>(c, f, 0, acc, (int)(n & 1));
    return launch_finalize<T, T>(f, c->stream);
}

static hipError_t launch_one(m2m_ctx* c, int64_t n, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    return c->prec == M2M_F64 ? launch_one_T<double>(c, n, e0, e1) : launch_one_T<float>(c, n, e0, e1);
}

template <typename T>
static hipError_t launch_prologue_T(m2m_ctx* c) {
    const int accum = c->prior.kind != M2M_PRIOR_FLAT ? 1 : 0;
    StepArgs<T, T> a;
    fill_step_args<T>(c, a, (int)(c->step & 1), 1, 0, accum);
    a.out = (T*)c->state[c->step & 1];   // observing only: the tags of the current state are written
    const Plan& p = c->plan;
    hipError_t e = launch_step<T, T>(a, c->pot_kind, c->sig, c->lay.nbin, p.ilp, p.nblock, p.threads, p.lds, c->stream);
    if (e != hipSuccess) return e;
    if (c->cells_apart && accum && (e = launch_cells_after<T>(c, (int)(c->step & 1))) != hipSuccess) return e;
    FinArgs<T, T> f;
    // the prologue's chi^2 shares are those of "step -1"
    fill_fin_args<T>(c, f, 1, accum, 1);
    return launch_finalize<T, T>(f, c->stream);
}

template <typename T>
static m2m_status derive_erange_T(m2m_ctx* c, std::vector<double>& er) {
    const Plan& p = c->plan;
    ErangeArgs<T> a;
    a.in = (const T*)c->state[0];
    a.stride = c->stride;
    a.tile_model = p.tile_model;
    a.tile_p0 = p.tile_p0;
    a.tile_cnt = p.tile_cnt;
    a.block_tile0 = p.block_tile0;
    a.block_slot0 = p.block_slot0;
    a.pots = (const Pot<double>*)c->pots64;
    a.out = p.erange_out;
    HIPCHK(c, launch_erange<T>(a, c->pot_kind, p.nblock, c->stream));
    std::vector<double> h((size_t)p.nslot * 2);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(h.data(), p.erange_out, h.size() * 8, hipMemcpyDeviceToHost));
    std::vector<int32_t> ms(c->M + 1);
    HIPCHK(c, hipMemcpy(ms.data(), p.model_slot, ms.size() * 4, hipMemcpyDeviceToHost));
    er.assign(2 * (size_t)c->M, 0.0);
    for (int m = 0; m < c->M; ++m) {
        double lo = INFINITY, hi = -INFINITY;
        for (int s = ms[m]; s < ms[m + 1]; ++s) { lo = std::min(lo, h[2 * s]); hi = std::max(hi, h[2 * s + 1]); }
        if (!(hi > lo)) hi = lo + 1e-6 * std::max(1.0, std::fabs(lo));
        er[2 * m] = lo;
        er[2 * m + 1] = hi;
    }
    return M2M_OK;
}

// ---------------------------------------------------------- host-side tables
// Potential parameters in precision X, and the circular-orbit energies
// E_c(r_k) = Phi(r_k) + r_k Phi'(r_k)/2 at kLcTab radii r_k = 1e-8 10^(16 k/(kLcTab-1))
// (equatorial plane; logarithmic and Hernquist + NFW models).
template <typename X>
static void build_tables(const m2m_ctx* c, std::vector<unsigned char>& pots, std::vector<X>& lctab) {
    pots.assign(sizeof(Pot<X>) * c->M, 0);
    lctab.assign((size_t)kLcTab * c->M, X(0));
    for (int m = 0; m < c->M; ++m) {
        const m2m_potential& q = c->pots[m];
        Pot<X> p{};
        p.kind = q.kind;
        p.lc_off = kLcTab * m;
        p.GM = (X)(q.G * q.M);
        p.a = (X)q.a;
        p.v2 = (X)(q.v0 * q.v0);
        p.Rc2 = (X)(q.Rc * q.Rc);
        p.iq2 = q.q > 0 ? (X)(1.0 / (q.q * q.q)) : X(0);
        p.GMh = q.kind == M2M_POT_HERNQUIST_NFW ? (X)(q.G * q.Mh) : X(0);
        p.rs = q.rs > 0 ? (X)q.rs : X(1);
        p.irs = q.rs > 0 ? (X)(1.0 / q.rs) : X(1);
        std::memcpy(pots.data() + sizeof(Pot<X>) * m, &p, sizeof(p));
        for (int k = 0; k < kLcTab; ++k) {
            const double r = 1e-8 * std::pow(10.0, 16.0 * k / (kLcTab - 1));
            double phi, d1;
            if (q.kind == M2M_POT_LOG) {
                const double s2 = q.Rc * q.Rc + r * r;
                phi = 0.5 * q.v0 * q.v0 * std::log(s2);
                d1 = q.v0 * q.v0 * r / s2;
            } else {
                phi = -q.G * q.M / (r + q.a);
                d1 = q.G * q.M / ((r + q.a) * (r + q.a));
                if (q.kind == M2M_POT_HERNQUIST_NFW && q.Mh > 0) {
                    const double l1 = std::log1p(r / q.rs);
                    phi += -q.G * q.Mh * l1 / r;
                    d1 += q.G * q.Mh * (l1 / (r * r) - 1.0 / (r * (r + q.rs)));
                }
            }
            lctab[(size_t)kLcTab * m + k] = (X)(phi + 0.5 * r * d1);
        }
    }
}

template <typename T>
static Layout<T> layout_of(const m2m_ctx* c) {
    Layout<T> L{};
    L.cosi = (T)std::cos(c->lay.incl);
    L.sini = (T)std::sin(c->lay.incl);
    L.nbin = c->lay.nbin;
    L.J = c->J;
    int off = 0, e0 = 0;
    for (int b = 0; b < c->lay.nbin; ++b) {
        const m2m_binning& d = c->lay.bin[b];
        BinDesc<T>& B = L.b[b];
        B.kind = d.kind;
        B.nmom = d.nmom;
        B.mom = 0;
        for (int k = 0; k < d.nmom; ++k) B.mom |= d.mom[k] << (kMomBits * k);
        B.off = off;
        B.edge0 = e0;
        B.gh0 = L.ngh;
        if (!c->gh_host[b].empty()) {
            L.has_gh = 1;
            L.ngh += (int)(c->gh_host[b].size() / 2);
        }
        if (d.kind == M2M_BIN_GRID) {
            B.nb = d.nx * d.ny;
            B.nx = d.nx;
            B.ny = d.ny;
            B.x0 = (T)d.x0;
            B.sx = (T)(d.nx / (d.x1 - d.x0));
            B.y0 = (T)d.y0;
            B.sy = (T)(d.ny / (d.y1 - d.y0));
            const double u = std::ldexp(1.0, -24), sx = d.nx / (d.x1 - d.x0), sy = d.ny / (d.y1 - d.y0);
            B.gx0 = (T)(2.0 * u * sx * std::fabs(d.x0));
            B.gy0 = (T)(2.0 * u * sy * std::fabs(d.y0));
            B.gys = (T)(6.0 * u * sy);
        } else {
            B.nb = d.nedge - 1;
            e0 += d.nedge;
            // log-spaced edges (as FP32 values): the kernels estimate the bin from
            // ln r when every edge lies within a quarter bin of its place
            if (sizeof(T) == 4 && d.nedge >= 3) {
                std::vector<double> lf(d.nedge);
                for (int k = 0; k < d.nedge; ++k) lf[k] = std::log((double)(float)c->edges_host[b][k]);
                const double x0 = (double)(float)lf[0], sx = (double)(float)((d.nedge - 1) / (lf[d.nedge - 1] - lf[0]));
                bool geo = std::isfinite(x0) && std::isfinite(sx) && sx > 0;
                for (int k = 0; geo && k < d.nedge; ++k) geo = std::fabs((lf[k] - x0) * sx - k) <= 0.25;
                if (geo) {
                    B.geo = 1;
                    B.x0 = (T)x0;
                    B.sx = (T)sx;
                }
            }
        }
        off += d.nmom * B.nb;
    }
    return L;
}

// Structure signature of the layout (selects kernels compiled for it).
static uint64_t signature_of(const m2m_ctx* c) {
    uint64_t code[kMaxBin] = {0, 0, 0, 0};
    for (int b = 0; b < c->lay.nbin; ++b) {
        const m2m_binning& d = c->lay.bin[b];
        int mom = 0;
        for (int k = 0; k < d.nmom; ++k) mom |= d.mom[k] << (kMomBits * k);
        code[b] = bin_code(d.kind, d.nmom, mom);
    }
    return layout_sig(c->lay.nbin, code[0], code[1], code[2], code[3]);
}

template <typename T>
static void build_layout(m2m_ctx* c) {
    const Layout<T> L = layout_of<T>(c);
    std::memcpy(c->lay_bytes, &L, sizeof(L));
    c->sig = signature_of(c);
    Cells C{};
    C.n0 = c->prior.n[0];
    C.n1 = c->prior.n[1];
    C.n2 = c->prior.n[2];
    C.ax2 = c->prior.ax2;
    C.ncell = c->NC;
    c->cells = C;
}

// Equatorial circular orbit of radius r (host, FP64): energy and angular momentum.
static void host_circular(const m2m_potential& q, double r, double* Ec, double* Lc) {
    double phi, d1;
    if (q.kind == M2M_POT_LOG) {
        const double s2 = q.Rc * q.Rc + r * r;
        phi = 0.5 * q.v0 * q.v0 * std::log(s2);
        d1 = q.v0 * q.v0 * r / s2;
    } else {
        phi = -q.G * q.M / (r + q.a);
        d1 = q.G * q.M / ((r + q.a) * (r + q.a));
        if (q.kind == M2M_POT_HERNQUIST_NFW && q.Mh > 0) {
            const double l1 = std::log1p(r / q.rs);
            phi += -q.G * q.Mh * l1 / r;
            d1 += q.G * q.Mh * (l1 / (r * r) - 1.0 / (r * (r + q.rs)));
        }
    }
    *Ec = phi + 0.5 * r * d1;
    *Lc = r * std::sqrt(std::max(0.0, r * d1));
}

// Lc(E) by bisection in ln r on [1e-8, 1e8] (end values outside the bracket);
// the circular radius goes to *rc when rc is given.
static double host_lc(const m2m_potential& q, double E, double* rc = nullptr) {
    double lo = std::log(1e-8), hi = std::log(1e8), Ec, Lc;
    host_circular(q, std::exp(lo), &Ec, &Lc);
    if (rc) *rc = 1e-8;
    if (E <= Ec) return Lc;
    host_circular(q, std::exp(hi), &Ec, &Lc);
    if (rc) *rc = 1e8;
    if (E >= Ec) return Lc;
    for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
        const double mid = 0.5 * (lo + hi);
        host_circular(q, std::exp(mid), &Ec, &Lc);
        if (Ec < E) lo = mid; else hi = mid;
    }
    if (rc) *rc = std::exp(0.5 * (lo + hi));
    host_circular(q, std::exp(0.5 * (lo + hi)), &Ec, &Lc);
    return Lc;
}

// Uniform-E table of Lc(E) for the FP32 kernels: kLcE pairs (ln Lc(E_k), bound)
// per model over [Emin - W/4, Emax + W/4] (W = Emax - Emin; kept below E = 0 for
// the bound-orbit potentials).  bound is a relative error bound of Lc from the
// FP32 linear interpolation of ln Lc on [E_k, E_k+1]: 4x the largest deviation
// from the FP64 value at three interior points, plus the effect of the FP32
// rounding of the index (2e-4 of the interval's change of ln Lc), of the energy
// (8e-7 times the largest |E| of the table, a few FP32 ulp) and of the table,
// interpolation and exponential (1e-6).  Beside it, ln r_c(E_k): the seeds of
// the FP64 Newton iteration that re-takes a cell decision left open.
template <typename T>
static m2m_status build_lc_etab(m2m_ctx* c, const std::vector<double>& er) {
    std::vector<float> tab(2 * (size_t)kLcE * c->M, 0.0f), rce((size_t)kLcE * c->M, 0.0f);
    c->lce_host.assign(2 * (size_t)c->M, 0.0f);
    std::vector<unsigned char> pots(sizeof(Pot<T>) * c->M);
    HIPCHK(c, hipMemcpy(pots.data(), c->pots_d, pots.size(), hipMemcpyDeviceToHost));
    for (int m = 0; m < c->M && c->prior.kind != M2M_PRIOR_FLAT; ++m) {
        const m2m_potential& q = c->pots[m];
        const double W = er[2 * m + 1] - er[2 * m];
        double lo = er[2 * m] - 0.25 * W, hi = er[2 * m + 1] + 0.25 * W;
        if (q.kind != M2M_POT_LOG && hi >= 0.0) hi = -1e-3 * std::fabs(er[2 * m]);
        if (!(hi > lo)) hi = lo + 1e-6;
        const double h = (hi - lo) / (kLcE - 1);
        std::vector<double> L(kLcE);
        for (int k = 0; k < kLcE; ++k) {
            double rc;
            L[k] = host_lc(q, lo + k * h, &rc);
            rce[(size_t)m * kLcE + k] = (float)std::log(rc);
        }
        for (int k = 0; k < kLcE; ++k) {
            double err = 1.0;
            if (k + 1 < kLcE && L[k] > 0 && L[k + 1] > 0) {
                const double l0 = std::log(L[k]), l1 = std::log(L[k + 1]);
                double dev = 0;
                for (double f : {0.25, 0.5, 0.75}) {
                    const double ex = host_lc(q, lo + (k + f) * h);
                    if (!(ex > 0)) { dev = 1.0; break; }
                    dev = std::max(dev, std::fabs(std::exp(l0 + f * (l1 - l0)) - ex) / ex);
                }
                // (the FP32 index, energy and evaluation errors are bounded per
                // particle by the kernel)
                err = std::min(1.0, 4.0 * dev + 1e-7);
            }
            tab[2 * ((size_t)m * kLcE + k)] = L[k] > 0 ? (float)std::log(L[k]) : -1e30f;
            tab[2 * ((size_t)m * kLcE + k) + 1] = (float)err;
        }
        Pot<T> p;
        std::memcpy(&p, pots.data() + sizeof(Pot<T>) * m, sizeof(p));
        p.lcE0 = (T)lo;
        p.lcEinv = (T)(1.0 / h);
        c->lce_host[2 * m] = (float)lo;
        c->lce_host[2 * m + 1] = (float)(1.0 / h);
        std::memcpy(pots.data() + sizeof(Pot<T>) * m, &p, sizeof(p));
    }
    HIPCHK(c, hipMemcpy(c->pots_d, pots.data(), pots.size(), hipMemcpyHostToDevice));
    m2m_status s = upload(c, (float**)&c->lcetab, tab);
    return s ? s : upload(c, (float**)&c->rcetab, rce);
}

// ------------------------------------------------------------------- create
// Bytes of one state buffer: 7 value rows and nbin + 1 tag rows.
static size_t state_bytes(const m2m_ctx* c) {
    return (size_t)c->stride * (7 * tsize(c) + sizeof(uint16_t) * (c->lay.nbin + 1));
}

template <typename T>
static m2m_status create_T(m2m_ctx* c, const m2m_target* tg, const void* xv, const void* w, int dev) {
    const int64_t N = c->N, S = c->stride;
    m2m_status s;
    if (state_bytes(c) >= ((size_t)1 << 32))
        return fail(c, M2M_ERR_UNSUPPORTED, "state buffer of " + std::to_string(state_bytes(c)) +
                                                " bytes: at most 4 GiB per context (split the particles)");
    for (int k = 0; k < 2; ++k) {
        if ((s = dalloc(c, (char**)&c->state[k], state_bytes(c)))) return s;
        HIPCHK(c, hipMemset(tags(c, k), 0xFF, state_bytes(c) - (size_t)7 * S * sizeof(T)));
    }
    // copy in and validate the weights and coordinates on the host
    std::vector<T> hx((size_t)6 * N), hw((size_t)N);
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    HIPCHK(c, hipMemcpy(hx.data(), xv, sizeof(T) * 6 * N, kind));
    HIPCHK(c, hipMemcpy(hw.data(), w, sizeof(T) * N, kind));
    for (int64_t i = 0; i < 6 * N; ++i)
        if (!std::isfinite((double)hx[i])) return fail(c, M2M_ERR_INVALID, "non-finite coordinate at " + std::to_string(i));
    for (int64_t i = 0; i < N; ++i)
        if (!(hw[i] > T(0)) || !std::isfinite((double)hw[i]))
            return fail(c, M2M_ERR_INVALID, "weights must be finite and > 0 (index " + std::to_string(i) + ")");
    for (int k = 0; k < 6; ++k)
        HIPCHK(c, hipMemcpy((T*)c->state[0] + k * S, hx.data() + k * N, sizeof(T) * N, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy((T*)c->state[0] + 6 * S, hw.data(), sizeof(T) * N, hipMemcpyHostToDevice));
    if (c->prior.kind != M2M_PRIOR_FLAT && (c->prior.period > 1 || c->prior.kind == M2M_PRIOR_MLP || c->cells_apart))
        if ((s = dalloc(c, (T**)&c->what, (size_t)S))) return s;
    if (c->prior.kind == M2M_PRIOR_MLP) {
        const m2m_prior& P = c->prior;
        c->mlp_nblk = (int)std::min<int64_t>(kMlpMaxInferBlocks, (N + kMlpInferThreads - 1) / kMlpInferThreads);
        if ((s = upload(c, &c->mlp_theta, c->mlp_init_host)) || (s = dalloc(c, &c->mlp_m, (size_t)kMlpNP)) ||
            (s = dalloc(c, &c->mlp_v, (size_t)kMlpNP)) || (s = dalloc(c, &c->mlp_sub, (size_t)P.mlp_subset)) ||
            (s = dalloc(c, &c->mlp_gpart, (size_t)(P.mlp_batch / kMlpSamples) * kMlpNP)) ||
            (s = dalloc(c, &c->mlp_red, 2 * (size_t)c->mlp_nblk)) || (s = dalloc(c, &c->mlp_stats, 8)))
            return s;
        HIPCHK(c, hipMemset(c->mlp_m, 0, sizeof(float) * kMlpNP));
        HIPCHK(c, hipMemset(c->mlp_v, 0, sizeof(float) * kMlpNP));
        HIPCHK(c, hipMemset(c->mlp_stats, 0, sizeof(double) * 8));
    }
    // tables (particle precision, and FP64 for the exact decisions)
    std::vector<unsigned char> pots, pots64;
    std::vector<T> lctab;
    std::vector<double> lctab64;
    build_tables<T>(c, pots, lctab);
    build_tables<double>(c, pots64, lctab64);
    if ((s = upload(c, (unsigned char**)&c->pots_d, pots)) || (s = upload(c, (T**)&c->lctab, lctab)) ||
        (s = upload(c, (unsigned char**)&c->pots64, pots64)) || (s = upload(c, &c->lctab64, lctab64)))
        return s;
    build_layout<T>(c);
    std::vector<T> ed;
    std::vector<double> ed64;
    for (int b = 0; b < c->lay.nbin; ++b)
        if (c->lay.bin[b].kind != M2M_BIN_GRID)
            for (double v : c->edges_host[b]) { ed.push_back((T)v); ed64.push_back(v); }
    if (ed.empty()) { ed.push_back(T(0)); ed64.push_back(0.0); }
    if ((s = upload(c, (T**)&c->edges, ed)) || (s = upload(c, &c->edges64, ed64))) return s;
    {
        // Gauss-Hermite (V, 1/sigma) pairs of the GH binnings, in layout order, in
        // the particle precision and in FP32 (the FP32 kernels' exact path)
        std::vector<T> gt;
        std::vector<float> gf;
        for (int b = 0; b < c->lay.nbin; ++b) {
            const std::vector<double>& g = c->gh_host[b];
            const size_t nb = g.size() / 2;
            for (size_t k = 0; k < nb; ++k) {
                gt.push_back((T)g[k]);
                gt.push_back((T)(1.0 / g[nb + k]));
                gf.push_back((float)g[k]);
                gf.push_back((float)(1.0 / g[nb + k]));
            }
        }
        if (gt.empty()) { gt.assign(2, T(0)); gf.assign(2, 0.0f); }
        if ((s = upload(c, (T**)&c->ghtab, gt)) || (s = upload(c, (float**)&c->ghtab32, gf))) return s;
    }
    std::vector<T> fw(c->M);
    for (int m = 0; m < c->M; ++m)
        fw[m] = (T)(c->prior.flat_value > 0 ? c->prior.flat_value : 1.0 / (double)(c->off[m + 1] - c->off[m]));
    if ((s = upload(c, (T**)&c->flatw, fw))) return s;
    const size_t MJ = (size_t)c->M * c->J;
    std::vector<double> Y(MJ), sg(MJ);
    for (int m = 0; m < c->M; ++m)
        for (int j = 0; j < c->J; ++j) {
            const size_t src = (tg->per_model ? (size_t)m * c->J : 0) + j;
            Y[(size_t)m * c->J + j] = tg->Y[src];
            sg[(size_t)m * c->J + j] = tg->sigma[src];
        }
    if ((s = upload(c, &c->Y, Y)) || (s = upload(c, &c->sigma, sg))) return s;
    if ((s = dalloc(c, &c->y, MJ)) || (s = dalloc(c, &c->ys, MJ)) || (s = dalloc(c, &c->delta, MJ)) ||
        (s = dalloc(c, (T**)&c->cvec, MJ)) || (s = dalloc(c, (T**)&c->cellmean, (size_t)c->M * std::max(1, c->NC))) ||
        (s = dalloc(c, &c->cellmean64, (size_t)c->M * std::max(1, c->NC))) ||
        (s = dalloc(c, &c->ring, (size_t)c->M * kRing)) || (s = dalloc(c, &c->flag, 1)) ||
        (s = dalloc(c, &c->bad_step, 1)) || (s = dalloc(c, &c->d_step, 2)))
        return s;
    // finalise column chunks (independent of the launch shape): kFinCols columns
    // of one model each; chi^2 shares double-buffered by step parity
    {
        std::vector<int32_t> cm, cc0, cn, mch(c->M + 1);
        for (int m = 0; m < c->M; ++m) {
            mch[m] = (int32_t)cm.size();
            for (int c0 = 0; c0 < c->pcols; c0 += kFinCols) {
                cm.push_back(m);
                cc0.push_back(c0);
                cn.push_back(std::min(kFinCols, c->pcols - c0));
            }
        }
        mch[c->M] = (int32_t)cm.size();
        c->nchunk = (int)cm.size();
        c->model_chunk_host = mch;
        c->chunk_model_host = cm;
        c->chunk_col0_host = cc0;
        c->chunk_ncol_host = cn;
        if ((s = upload(c, &c->model_chunk, mch)) || (s = dalloc(c, &c->chunk_chi, 4 * (size_t)c->nchunk)))
            return s;
        HIPCHK(c, hipMemset(c->chunk_chi, 0, sizeof(double) * 4 * c->nchunk));
    }
    HIPCHK(c, hipMemset(c->flag, 0, sizeof(int)));
    HIPCHK(c, hipMemset(c->bad_step, 0, sizeof(long long)));
    HIPCHK(c, hipMemset(c->d_step, 0, 2 * sizeof(long long)));
    HIPCHK(c, hipMemset(c->ring, 0, sizeof(StatRow) * (size_t)c->M * kRing));
    HIPCHK(c, hipMemset(c->cvec, 0, sizeof(T) * MJ));
    HIPCHK(c, hipMemset(c->cellmean, 0, sizeof(T) * (size_t)c->M * std::max(1, c->NC)));
    HIPCHK(c, hipMemset(c->cellmean64, 0, sizeof(double) * (size_t)c->M * std::max(1, c->NC)));
    if (c->mp) {
        // node radii (FP64, the interval decisions), node table, interval sums,
        // readback tables
        const m2m_potential& q = c->mp_pot;
        const int nn = q.nnode, nlm = (q.lmax + 1) * (q.lmax + 1);
        const double lr0 = std::log(q.rmin), dl = (std::log(q.rmax) - lr0) / (nn - 1);
        std::vector<double> rk(nn);
        for (int k = 0; k < nn; ++k) rk[k] = std::exp(lr0 + k * dl);
        const size_t ntab = (size_t)nn * (sizeof(T) == 4 ? kMpRowF : kMpW);
        if ((s = upload(c, &c->mp_rk, rk)) || (s = dalloc(c, (T**)&c->mp_tab, ntab)) ||
            (s = dalloc(c, &c->mp_S, (size_t)(nn + 1) * kMpW)) || (s = dalloc(c, &c->mp_A64, (size_t)nn * nlm)) ||
            (s = dalloc(c, &c->mp_B64, (size_t)nn * nlm)) || (s = dalloc(c, (T**)&c->mp_acc[0], 3 * (size_t)c->stride)) ||
            (s = dalloc(c, (T**)&c->mp_acc[1], 3 * (size_t)c->stride)))
            return s;
        HIPCHK(c, hipMemset(c->mp_tab, 0, sizeof(T) * ntab));
        HIPCHK(c, hipMemset(c->mp_S, 0, sizeof(double) * (nn + 1) * kMpW));
        if (sizeof(T) == 4) {
            // counting sort by interval: G blocks of R particles (G <= 1024)
            c->mp_G = (int)std::min<int64_t>(1024, (N + kMpSortThreads - 1) / kMpSortThreads);
            c->mp_R = ((N + c->mp_G - 1) / c->mp_G + kMpSortThreads - 1) / kMpSortThreads * kMpSortThreads;
            c->mp_maxchunk = (int)((N + kMpChunk - 1) / kMpChunk + nn + 1);
            const size_t nk = (size_t)(nn + 1) * c->mp_G;
            if ((s = dalloc(c, &c->mp_key, (size_t)N)) || (s = dalloc(c, &c->mp_counts, nk)) ||
                (s = dalloc(c, &c->mp_offs, nk)) || (s = dalloc(c, &c->mp_total, (size_t)nn + 1)) ||
                (s = dalloc(c, &c->mp_sorted, (size_t)N)) ||
                (s = dalloc(c, &c->mp_part, (size_t)c->mp_maxchunk * kMpW)))
                return s;
        }
    }
    // launch plan, energy range of the prior grid, prologue observe
    if ((s = make_plan(c, c->launch.threads, c->launch.ilp, c->launch.blocks_per_cu))) return s;
    std::vector<double> er(2 * (size_t)c->M, 0.0);
    if (c->prior.kind != M2M_PRIOR_FLAT) {
        if (!c->erange_user.empty()) er = c->erange_user;
        else if ((s = derive_erange_T<T>(c, er))) return s;
    }
    c->erange_host = er;
    std::vector<T> erT(er.size());
    for (size_t k = 0; k < er.size(); ++k) erT[k] = (T)er[k];
    if ((s = upload(c, (T**)&c->erange, erT)) || (s = upload(c, &c->erange64, er))) return s;
    if ((s = build_lc_etab<T>(c, er)) || (s = upload_exact(c))) return s;
    if (c->mp) {
        // coefficients of the initial state and its field (the first kick of step 0)
        MpArgs<T> mp;
        fill_mp_args<T>(c, mp, c->state[0], 1, 2);
        HIPCHK(c, launch_mp_build<T>(mp, c->plan.nblock, c->mp_lds, c->stream));
    }
    HIPCHK(c, launch_prologue_T<T>(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return M2M_OK;
}

extern "C" int32_t m2m_abi_version(void) { return M2M_ABI_VERSION; }

extern "C" m2m_status m2m_create(const m2m_config* cfg, const m2m_obs_layout* layout, const m2m_target* target,
                                 const void* xv, const void* w, int32_t device_ptrs, m2m_ctx** out) {
    if (!out) return fail(nullptr, M2M_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!xv || !w) return fail(nullptr, M2M_ERR_INVALID, "particle arrays missing");
    int64_t N = 0;
    int J = 0;
    m2m_status s = validate(cfg, layout, target, &N, &J);
    if (s) return s;
    if (!device_ptrs) {
        // host inputs are checked before any device work
        const bool f64 = cfg->precision == M2M_F64;
        for (int64_t i = 0; i < 6 * N; ++i) {
            const double v = f64 ? ((const double*)xv)[i] : ((const float*)xv)[i];
            if (!std::isfinite(v)) return fail(nullptr, M2M_ERR_INVALID, "non-finite coordinate at " + std::to_string(i));
        }
        for (int64_t i = 0; i < N; ++i) {
            const double v = f64 ? ((const double*)w)[i] : ((const float*)w)[i];
            if (!(v > 0) || !std::isfinite(v))
                return fail(nullptr, M2M_ERR_INVALID, "weights must be finite and > 0 (index " + std::to_string(i) + ")");
        }
    }
    m2m_ctx* c = new m2m_ctx();
    c->prec = cfg->precision;
    c->update = cfg->update;
    c->frozen = cfg->frozen ? 1 : 0;
    c->dt = cfg->dt;
    c->eps = cfg->eps;
    c->mu = cfg->mu;
    c->tau = cfg->tau;
    c->M = cfg->n_models;
    c->off.assign(cfg->model_offsets, cfg->model_offsets + c->M + 1);
    c->pots.assign(cfg->potentials, cfg->potentials + c->M);
    if (c->pots[0].kind == M2M_POT_MULTIPOLE) {
        // the self-consistent model: energies of the prior cells are measured in
        // the analytic reference potential (a flat prior needs none)
        c->mp = true;
        c->mp_pot = c->pots[0];
        if (cfg->prior.ref.kind >= 0) {
            c->pots[0] = cfg->prior.ref;
        } else {
            c->pots[0] = m2m_potential{};
            c->pots[0].kind = M2M_POT_HERNQUIST;
            c->pots[0].G = c->pots[0].M = c->pots[0].a = 1.0;
        }
    }
    c->pot_kind = c->pots[0].kind;
    c->prior = cfg->prior;
    if (cfg->prior.Erange) c->erange_user.assign(cfg->prior.Erange, cfg->prior.Erange + 2 * (size_t)c->M);
    c->prior.Erange = nullptr;
    if (cfg->prior.kind == M2M_PRIOR_MLP) c->mlp_init_host.assign(cfg->prior.mlp_init, cfg->prior.mlp_init + M2M_MLP_NPARAM);
    c->prior.mlp_init = nullptr;
    c->lay = *layout;
    for (int b = 0; b < layout->nbin; ++b) {
        const m2m_binning& d = layout->bin[b];
        if (d.kind != M2M_BIN_GRID) c->edges_host[b].assign(d.edges, d.edges + d.nedge);
        c->lay.bin[b].edges = nullptr;
        bool gh = false;
        for (int k = 0; k < d.nmom; ++k) gh |= d.mom[k] >= M2M_MOM_H1;
        if (gh) {
            const int nb = d.kind == M2M_BIN_GRID ? d.nx * d.ny : d.nedge - 1;
            c->gh_host[b].assign(d.gh, d.gh + 2 * (size_t)nb);
        }
        c->lay.bin[b].gh = nullptr;
    }
    c->nedge = 0;
    c->ngh = 0;
    for (int b = 0; b < layout->nbin; ++b) {
        c->nedge += (int)c->edges_host[b].size();
        c->ngh += (int)(c->gh_host[b].size() / 2);
    }
    c->N = N;
    c->stride = (N + 63) / 64 * 64;
    c->J = J;
    c->JP = (J + 1) & ~1;
    c->NC = cfg->prior.kind == M2M_PRIOR_FLAT ? 0 : cfg->prior.n[0] * cfg->prior.n[1] * cfg->prior.n[2];
    c->pcols = c->JP + 2 * c->NC;
    c->stream = (hipStream_t)cfg->stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->numCU, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
    if (e == hipSuccess) {
        // the static scratch of the allocation-free entry point: its device
        // address, looked up once per device (with the device current); a failed
        // lookup disables that entry point only
        const hipError_t es = mlp_noalloc_scratch(c->device, &c->noalloc_scratch);
        if (es != hipSuccess) {
            (void)hipGetLastError();
            c->noalloc_scratch = nullptr;
            c->noalloc_error = std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(es);
        }
    }
    if (e == hipSuccess && !c->stream) {
        // the legacy default stream cannot be captured into graphs: run on a
        // stream of our own (default priority) unless the caller names one
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        c->own_stream = e == hipSuccess;
    }
    if (e != hipSuccess) {
        delete c;
        return fail(nullptr, M2M_ERR_DEVICE, std::string("no usable HIP device: ") + hipGetErrorString(e));
    }
    c->launch.threads = c->prec == M2M_F64 ? 256 : 1024;
    c->launch.ilp = 1;
    c->launch.blocks_per_cu = 1;
    c->launch.graph_steps = 0;
    c->launch.timing = 0;
    const size_t lds_need = 160 * 1024;
    {
        // LDS of the fused kernel with the prior cells (as make_plan computes it)
        const int NCe = (c->NC + 1) & ~1, NE = (c->nedge + 1) & ~1;
        const size_t fused = 8 * ((size_t)c->JP + kTrash + c->NC + kTrash + NE + 2 + 64) +
                             4 * ((size_t)NCe + kTrash) + 4 * ((size_t)c->JP + 2 + NCe + NE + kLcTab) +
                             (c->NC > 0 ? 8 * (size_t)kLcE : 0) + 8 * (size_t)kFixQ * 16 + 8 * (size_t)c->ngh;
        // the learned prior's judge grid, and FP32 histogram priors too large for
        // the fused kernel, are accumulated by the cell kernel
        c->cells_apart = c->prec == M2M_F32 && (c->prior.kind == M2M_PRIOR_MLP ||
                                                (c->prior.kind == M2M_PRIOR_HIST && fused > (size_t)c->max_lds));
    }
    if (c->cells_apart) {
        const int NCe = (c->NC + 1) & ~1;
        c->cells_lds = 8 * (size_t)c->NC + 8 * (size_t)kLcE + 4 * (size_t)NCe;
        if (c->cells_lds > (size_t)c->max_lds) {
            const std::string why = "prior grid of " + std::to_string(c->NC) + " cells needs " +
                                    std::to_string(c->cells_lds) + " bytes of LDS (max " + std::to_string(c->max_lds) + ")";
            m2m_destroy(c);
            return fail(nullptr, M2M_ERR_UNSUPPORTED, why);
        }
        (void)set_cells_lds_limit(lds_need);
    }
    if (c->prec == M2M_F64) {
        (void)set_step_lds_limit<double, double>(c->pot_kind, lds_need);
        if (c->mp) (void)set_mp_lds_limit<double, double>(lds_need);
    } else {
        (void)set_step_lds_limit<float, float>(c->pot_kind, lds_need);
        if (c->mp) (void)set_mp_lds_limit<float, float>(lds_need);
    }
    (void)hipGetLastError();
    s = c->prec == M2M_F64 ? create_T<double>(c, target, xv, w, device_ptrs)
                           : create_T<float>(c, target, xv, w, device_ptrs);
    if (s) {
        g_create_error = c->msg;
        m2m_destroy(c);
        return s;
    }
    *out = c;
    return M2M_OK;
}

// --------------------------------------------------------------------- step
static m2m_status sticky(m2m_ctx* c) {
    if (c->status == M2M_ERR_NONPOSITIVE_WEIGHT || c->status == M2M_ERR_NONFINITE || c->status == M2M_ERR_DEVICE)
        return c->status;
    return M2M_OK;
}

static m2m_status check_flag(m2m_ctx* c, int64_t start) {
    int flag = 0;
    long long bad = 0;
    HIPCHK(c, hipMemcpy(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (!flag) return M2M_OK;
    HIPCHK(c, hipMemcpy(&bad, c->bad_step, sizeof(long long), hipMemcpyDeviceToHost));
    c->step = bad;
    c->status = (flag & 2) ? M2M_ERR_NONFINITE : M2M_ERR_NONPOSITIVE_WEIGHT;
    (void)start;
    return fail(c, c->status, std::string(flag & 2 ? "non-finite weight" : "non-positive weight") +
                                  " produced by the update of step " + std::to_string(bad) +
                                  "; the context holds the state at the start of that step");
}

// HIP graphs are used when the step sequence is the same every step (flat prior
// or a moving prior refreshed every step) and no per-kernel timing is asked for
// (event records inside a graph cannot be timed).
static bool graphable(const m2m_ctx* c) {
    return c->launch.graph_steps > 0 && !c->launch.timing &&
           (c->prior.kind == M2M_PRIOR_FLAT || (c->prior.kind == M2M_PRIOR_HIST && c->prior.period == 1));
}

// Capture K steps (K even, so a replay ends on the buffer parity it started on).
static m2m_status build_graph(m2m_ctx* c, int parity) {
    const int K = (c->launch.graph_steps + 1) & ~1;
    if (c->graph[parity]) { (void)hipGraphExecDestroy(c->graph[parity]); c->graph[parity] = nullptr; }
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < K && e == hipSuccess; ++k) e = launch_one(c, parity + k);
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, M2M_ERR_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&c->graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, M2M_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    c->graph_k[parity] = K;
    return M2M_OK;
}

extern "C" m2m_status m2m_step(m2m_ctx* c, int64_t n_steps, m2m_step_stats* last) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (m2m_status s = sticky(c)) return s;
    if (n_steps < 0) return fail(c, M2M_ERR_INVALID, "n_steps < 0");
    const int64_t start = c->step;
    int64_t left = n_steps;
    c->last_launches = 0;
    c->last_kernel_ms = 0;
    if (graphable(c)) {
        const int K = (c->launch.graph_steps + 1) & ~1;
        while (left >= K) {
            const int par = (int)(c->step & 1);
            if (!c->graph[par] || c->graph_k[par] != K)
                if (m2m_status s = build_graph(c, par)) return s;
            HIPCHK(c, hipGraphLaunch(c->graph[par], c->stream));
            c->step += K;
            left -= K;
        }
    }
    if (c->launch.timing && left > 0) {
        const int64_t nt = std::min<int64_t>(left, 4096);
        if ((int64_t)c->events.size() < 2 * nt) {
            while ((int64_t)c->events.size() < 2 * nt) {
                hipEvent_t ev;
                HIPCHK(c, hipEventCreate(&ev));
                c->events.push_back(ev);
            }
        }
        for (int64_t k = 0; k < left; ++k) {
            hipEvent_t e0 = k < nt ? c->events[2 * k] : nullptr, e1 = k < nt ? c->events[2 * k + 1] : nullptr;
            HIPCHK(c, launch_one(c, c->step, e0, e1));
            ++c->step;
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double tot = 0;
        for (int64_t k = 0; k < nt; ++k) {
            float ms = 0;
            HIPCHK(c, hipEventElapsedTime(&ms, c->events[2 * k], c->events[2 * k + 1]));
            tot += ms;
        }
        c->last_kernel_ms = tot / nt;
        c->last_launches = nt;
        left = 0;
    }
    for (; left > 0; --left) {
        HIPCHK(c, launch_one(c, c->step));
        ++c->step;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (m2m_status s = check_flag(c, start)) return s;
    if (last && c->step > 0) {
        const int64_t row = (c->step - 1) % kRing;
        for (int m = 0; m < c->M; ++m) {
            StatRow r;
            HIPCHK(c, hipMemcpy(&r, c->ring + (size_t)m * kRing + row, sizeof(r), hipMemcpyDeviceToHost));
            std::memcpy(&last[m], &r, sizeof(r));
        }
    }
    return M2M_OK;
}

extern "C" int64_t m2m_step_index(const m2m_ctx* c) { return c ? c->step : -1; }

// ---------------------------------------------------------------- readbacks
extern "C" m2m_status m2m_observables(m2m_ctx* c, int32_t model, double* y, double* ys, double* delta, double* chi2) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (model < 0 || model >= c->M) return fail(c, M2M_ERR_INVALID, "model out of range");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const size_t o = (size_t)model * c->J, n = sizeof(double) * c->J;
    if (y) HIPCHK(c, hipMemcpy(y, c->y + o, n, hipMemcpyDeviceToHost));
    if (ys) HIPCHK(c, hipMemcpy(ys, c->ys + o, n, hipMemcpyDeviceToHost));
    if (delta) HIPCHK(c, hipMemcpy(delta, c->delta + o, n, hipMemcpyDeviceToHost));
    if (chi2) {
        // chi^2 of the current state: the model's shares from the last finalise
        const int par = (int)((c->step + 1) & 1);
        std::vector<double> sh(2 * (size_t)c->nchunk);
        HIPCHK(c, hipMemcpy(sh.data(), c->chunk_chi + 2 * (size_t)par * c->nchunk, sizeof(double) * sh.size(),
                            hipMemcpyDeviceToHost));
        double x2 = 0;
        for (int k = c->model_chunk_host[model]; k < c->model_chunk_host[model + 1]; ++k) x2 += sh[2 * k];
        *chi2 = x2;
    }
    return M2M_OK;
}

static m2m_status copy_rows(m2m_ctx* c, void* dst, int row0, int nrow, int dev) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const size_t ts = tsize(c);
    const char* src = (const char*)c->state[c->step & 1];
    for (int k = 0; k < nrow; ++k)
        HIPCHK(c, hipMemcpy((char*)dst + (size_t)k * c->N * ts, src + (size_t)(row0 + k) * c->stride * ts, c->N * ts,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return M2M_OK;
}

extern "C" m2m_status m2m_weights(m2m_ctx* c, void* w_out, int32_t device_ptr) {
    if (!c || !w_out) return fail(c, M2M_ERR_INVALID, "null argument");
    return copy_rows(c, w_out, 6, 1, device_ptr);
}

extern "C" m2m_status m2m_particles(m2m_ctx* c, void* xv_out, int32_t device_ptr) {
    if (!c || !xv_out) return fail(c, M2M_ERR_INVALID, "null argument");
    return copy_rows(c, xv_out, 0, 6, device_ptr);
}

extern "C" m2m_status m2m_tags(m2m_ctx* c, uint16_t* out, int32_t device_ptr) {
    if (!c || !out) return fail(c, M2M_ERR_INVALID, "null argument");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const uint16_t* src = tags(c, (int)(c->step & 1));
    for (int k = 0; k <= c->lay.nbin; ++k)
        HIPCHK(c, hipMemcpy(out + (size_t)k * c->N, src + (size_t)k * c->stride, sizeof(uint16_t) * c->N,
                            device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return M2M_OK;
}

template <typename T>
static m2m_status gather_T(m2m_ctx* c, void* out, int dev) {
    if (!c->scratch_n) {
        if (m2m_status s = dalloc(c, (T**)&c->scratch_n, (size_t)c->stride)) return s;
    }
    int wm, acc;
    prior_modes(c, c->step, &wm, &acc);
    if (wm == 2) wm = 1;   // a refresh step would compute the table priors
    HIPCHK(c, launch_gather<T>(gather_args<T>(c, (int)(c->step & 1), wm, (T*)c->scratch_n), c->pot_kind,
                               c->plan.nblock, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(out, c->scratch_n, sizeof(T) * c->N, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return M2M_OK;
}

extern "C" m2m_status m2m_priors(m2m_ctx* c, void* what_out, double* cell_mean, int32_t device_ptr) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (what_out) {
        m2m_status s = c->prec == M2M_F64 ? gather_T<double>(c, what_out, device_ptr) : gather_T<float>(c, what_out, device_ptr);
        if (s) return s;
    }
    if (cell_mean) {
        if (c->NC == 0) return fail(c, M2M_ERR_INVALID, "flat prior has no cell table");
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipMemcpy(cell_mean, c->cellmean64, sizeof(double) * c->M * c->NC, hipMemcpyDeviceToHost));
    }
    return M2M_OK;
}

extern "C" m2m_status m2m_history(m2m_ctx* c, m2m_step_stats* out, int64_t max_rows, int64_t* n_rows) {
    if (!c || !out || !n_rows || max_rows < 0) return fail(c, M2M_ERR_INVALID, "null argument");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int64_t have = std::min<int64_t>(c->step, kRing);
    const int64_t per = std::min<int64_t>(have, max_rows / c->M);
    std::vector<StatRow> ring((size_t)c->M * kRing);
    HIPCHK(c, hipMemcpy(ring.data(), c->ring, sizeof(StatRow) * ring.size(), hipMemcpyDeviceToHost));
    int64_t k = 0;
    for (int64_t s = c->step - per; s < c->step; ++s)
        for (int m = 0; m < c->M; ++m) std::memcpy(&out[k++], &ring[(size_t)m * kRing + s % kRing], sizeof(StatRow));
    *n_rows = k;
    return M2M_OK;
}

// ------------------------------------------------------ potential sequence
extern "C" m2m_status m2m_delta_chi2(m2m_ctx* c, double* chi2, double* delta, int32_t* best) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (c->step < 1) return fail(c, M2M_ERR_INVALID, "no step taken yet");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int64_t row = (c->step - 1) % kRing;
    std::vector<double> x(c->M);
    for (int m = 0; m < c->M; ++m) {
        StatRow r;
        HIPCHK(c, hipMemcpy(&r, c->ring + (size_t)m * kRing + row, sizeof(r), hipMemcpyDeviceToHost));
        x[m] = r.chi2;
    }
    int b = 0;
    for (int m = 1; m < c->M; ++m)
        if (x[m] < x[b]) b = m;
    for (int m = 0; m < c->M; ++m) {
        if (chi2) chi2[m] = x[m];
        if (delta) delta[m] = x[m] - x[b];
    }
    if (best) *best = b;
    return M2M_OK;
}

// ------------------------------------------------------------------ tracers
template <typename T>
static m2m_status set_tracers_T(m2m_ctx* c, const m2m_tracers* t) {
    const int n = t->n, nb = c->trc_nb;
    // CSR by bin (stable), the caller's order kept in perm
    std::vector<int32_t> first(nb + 1, 0), order(n), tbin(n);
    for (int k = 0; k < n; ++k) first[t->bin[k] + 1] += 1;
    for (int b = 0; b < nb; ++b) first[b + 1] += first[b];
    std::vector<int32_t> fill(first.begin(), first.end() - 1);
    c->trc_perm.assign(n, 0);
    for (int k = 0; k < n; ++k) {
        const int pos = fill[t->bin[k]]++;
        order[pos] = k;
        c->trc_perm[k] = pos;
    }
    std::vector<T> V(n), is(n), nf(n);
    for (int q = 0; q < n; ++q) {
        const int k = order[q];
        tbin[q] = t->bin[k];
        V[q] = (T)t->v[k];
        is[q] = (T)(1.0 / t->width[k]);
        nf[q] = (T)(1.0 / (std::sqrt(2.0 * M_PI) * t->width[k]));
    }
    c->trc_nblk = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(kTrcBlocks, c->numCU), (c->N + 1023) / 1024));
    m2m_status s;
    if ((s = upload(c, &c->trc_first, first)) || (s = upload(c, &c->trc_tbin, tbin)) ||
        (s = upload(c, (T**)&c->trc_V, V)) || (s = upload(c, (T**)&c->trc_is, is)) ||
        (s = upload(c, (T**)&c->trc_nf, nf)) || (s = dalloc(c, (T**)&c->trc_cL, (size_t)n)) ||
        (s = dalloc(c, (T**)&c->trc_cM, (size_t)nb)) || (s = dalloc(c, (T**)&c->trc_extra, (size_t)c->stride)) ||
        (s = dalloc(c, &c->trc_part, (size_t)c->trc_nblk * (n + nb))) ||
        (s = dalloc(c, &c->trc_Ls, (size_t)n)) ||
        (s = dalloc(c, &c->trc_Ms, (size_t)nb)) || (s = dalloc(c, &c->trc_ll, 1)))
        return s;
    c->trc_lambda = t->lambda;
    c->trc_n = n;
    const TracerArgs<T> a = tracer_args<T>(c, 0, 1);
    const size_t lds = tracer_lds<T>(a);
    if (lds > (size_t)c->max_lds) {
        c->trc_n = 0;
        return fail(c, M2M_ERR_UNSUPPORTED, "tracers need " + std::to_string(lds) + " bytes of LDS per block");
    }
    HIPCHK(c, set_tracer_lds_limit<T>(lds));
    // the initial state's sums start the smoothing
    HIPCHK(c, launch_tracer_observe<T>(a, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return M2M_OK;
}

extern "C" m2m_status m2m_set_tracers(m2m_ctx* c, const m2m_tracers* t) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (!t || !t->bin || !t->v || !t->width) return fail(c, M2M_ERR_INVALID, "null argument");
    if (c->M != 1 || c->mp || c->prior.kind == M2M_PRIOR_MLP)
        return fail(c, M2M_ERR_UNSUPPORTED, "tracers need a single-model context with an analytic potential "
                                            "and no learned prior");
    if (c->trc_n) return fail(c, M2M_ERR_INVALID, "tracers are already set");
    if (c->step != 0) return fail(c, M2M_ERR_INVALID, "tracers must be set before the first step");
    if (t->binning < 0 || t->binning >= c->lay.nbin) return fail(c, M2M_ERR_INVALID, "binning index out of range");
    if (t->n < 1 || t->n > M2M_TRACERS_MAX) return fail(c, M2M_ERR_INVALID, "n must be in [1, 4096]");
    if (!is_fin(t->lambda)) return fail(c, M2M_ERR_INVALID, "lambda must be finite");
    const m2m_binning& d = c->lay.bin[t->binning];
    const int nb = d.kind == M2M_BIN_GRID ? d.nx * d.ny : d.nedge - 1;
    for (int k = 0; k < t->n; ++k) {
        if (t->bin[k] < 0 || t->bin[k] >= nb) return fail(c, M2M_ERR_INVALID, "tracer bin out of range");
        if (!is_fin(t->v[k])) return fail(c, M2M_ERR_INVALID, "tracer velocities must be finite");
        if (!(t->width[k] > 0.0) || !is_fin(t->width[k])) return fail(c, M2M_ERR_INVALID, "widths must be > 0");
    }
    if (c->status == M2M_ERR_DEVICE) return c->status;
    c->trc_binning = t->binning;
    c->trc_nb = nb;
    return c->prec == M2M_F64 ? set_tracers_T<double>(c, t) : set_tracers_T<float>(c, t);
}

extern "C" m2m_status m2m_tracer_state(m2m_ctx* c, double* loglike, double* L, double* M) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (!c->trc_n) return fail(c, M2M_ERR_INVALID, "the context has no tracers");
    if (loglike) {
        const hipError_t e = c->prec == M2M_F64 ? launch_tracer_loglike<double>(tracer_args<double>(c, 0, 0), c->stream)
                                                : launch_tracer_loglike<float>(tracer_args<float>(c, 0, 0), c->stream);
        HIPCHK(c, e);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (loglike) HIPCHK(c, hipMemcpy(loglike, c->trc_ll, sizeof(double), hipMemcpyDeviceToHost));
    if (L) {
        std::vector<double> Ls(c->trc_n);
        HIPCHK(c, hipMemcpy(Ls.data(), c->trc_Ls, sizeof(double) * c->trc_n, hipMemcpyDeviceToHost));
        for (int k = 0; k < c->trc_n; ++k) L[k] = Ls[c->trc_perm[k]];
    }
    if (M) HIPCHK(c, hipMemcpy(M, c->trc_Ms, sizeof(double) * c->trc_nb, hipMemcpyDeviceToHost));
    return M2M_OK;
}

// ------------------------------------------------------------ shell moments
extern "C" m2m_status m2m_shell_moments(m2m_ctx* c, int32_t model, const double* edges, int32_t nshell, double* out) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (!edges || !out) return fail(c, M2M_ERR_INVALID, "null argument");
    if (model < 0 || model >= c->M) return fail(c, M2M_ERR_INVALID, "model index out of range");
    if (nshell < 1 || nshell > kShellMax) return fail(c, M2M_ERR_INVALID, "nshell must be in [1, 256]");
    if (!(edges[0] > 0.0) || !is_fin(edges[nshell])) return fail(c, M2M_ERR_INVALID, "edges must be finite and > 0");
    for (int k = 0; k < nshell; ++k)
        if (!(edges[k + 1] > edges[k])) return fail(c, M2M_ERR_INVALID, "edges must increase strictly");
    if (c->status == M2M_ERR_DEVICE) return c->status;
    const size_t npart = (size_t)kShellBlocks * 4 * kShellMax;
    if (!c->shell_buf)
        if (m2m_status s = dalloc(c, &c->shell_buf, npart + (kShellMax + 1) + 4 * kShellMax)) return s;
    double* d_edges = c->shell_buf + npart;
    double* d_out = d_edges + (kShellMax + 1);
    HIPCHK(c, hipMemcpyAsync(d_edges, edges, sizeof(double) * (nshell + 1), hipMemcpyHostToDevice, c->stream));
    const int64_t p0 = c->off[model], p1 = c->off[model + 1];
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kShellBlocks, (p1 - p0 + kShellThreads - 1) / kShellThreads));
    if (c->prec == M2M_F64) {
        ShellArgs<double> a{(const double*)c->state[c->step & 1], c->stride, p0, p1, d_edges, nshell, c->shell_buf};
        HIPCHK(c, launch_shell_moments<double>(a, blocks, d_out, c->stream));
    } else {
        ShellArgs<float> a{(const float*)c->state[c->step & 1], c->stride, p0, p1, d_edges, nshell, c->shell_buf};
        HIPCHK(c, launch_shell_moments<float>(a, blocks, d_out, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(out, d_out, sizeof(double) * 4 * nshell, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return M2M_OK;
}

// --------------------------------------------------------- multipole tables
extern "C" m2m_status m2m_multipole_tables(m2m_ctx* c, double* A, double* B) {
    if (!c || !A || !B) return fail(c, M2M_ERR_INVALID, "null argument");
    if (!c->mp) return fail(c, M2M_ERR_INVALID, "the context's model has no multipole potential");
    if (c->status == M2M_ERR_DEVICE) return c->status;
    const size_t n = (size_t)c->mp_pot.nnode * (c->mp_pot.lmax + 1) * (c->mp_pot.lmax + 1);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(A, c->mp_A64, n * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(B, c->mp_B64, n * sizeof(double), hipMemcpyDeviceToHost));
    return M2M_OK;
}

// ------------------------------------------------------------ learned prior
extern "C" m2m_status m2m_mlp_state(m2m_ctx* c, float* theta, double* judge, int32_t* used_fallback,
                                    int64_t* refreshes) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (c->prior.kind != M2M_PRIOR_MLP) return fail(c, M2M_ERR_INVALID, "the context has no learned prior");
    if (c->status == M2M_ERR_DEVICE) return c->status;
    double st[8];
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(st, c->mlp_stats, sizeof(st), hipMemcpyDeviceToHost));
    if (theta) HIPCHK(c, hipMemcpy(theta, c->mlp_theta, sizeof(float) * kMlpNP, hipMemcpyDeviceToHost));
    if (judge) *judge = st[4];
    if (used_fallback) *used_fallback = st[5] != 0.0;
    if (refreshes) *refreshes = (int64_t)st[6];
    return M2M_OK;
}

extern "C" m2m_status m2m_mlp_loss_grad(m2m_ctx* c, const float* theta, const float* samples, int32_t n, float* grad,
                                        double* loss) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (c->prior.kind != M2M_PRIOR_MLP) return fail(c, M2M_ERR_INVALID, "the context has no learned prior");
    if (!theta || !samples || !grad) return fail(c, M2M_ERR_INVALID, "null argument");
    if (n < kMlpSamples || n % kMlpSamples) return fail(c, M2M_ERR_INVALID, "n must be a positive multiple of 32");
    if (m2m_status s = sticky(c)) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // scratch of this call only: parameters, samples, partial rows, gradient, loss terms
    const size_t nblk = (size_t)n / kMlpSamples;
    float *th = nullptr, *gp = nullptr, *gr = nullptr, *ls = nullptr;
    float4* sm = nullptr;
    m2m_status s;
    if ((s = dalloc(c, &th, (size_t)kMlpNP)) || (s = dalloc(c, &sm, (size_t)n)) || (s = dalloc(c, &gp, nblk * kMlpNP)) ||
        (s = dalloc(c, &gr, (size_t)kMlpNP)) || (s = dalloc(c, &ls, (size_t)n))) {
        for (void* q : {(void*)th, (void*)sm, (void*)gp, (void*)gr, (void*)ls}) dfree(c, q);
        return s;
    }
    MlpArgs a{};
    fill_mlp_args(c, a, c->step);
    a.theta = th;
    a.sub = sm;
    a.gpart = gp;
    a.batch = n;
    a.loss = ls;
    std::vector<float> hl((size_t)n);
    hipError_t e = hipMemcpy(th, theta, sizeof(float) * kMlpNP, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sm, samples, sizeof(float) * 4 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_mlp_grad(a, gr, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(grad, gr, sizeof(float) * kMlpNP, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(hl.data(), ls, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost);
    for (void* q : {(void*)th, (void*)sm, (void*)gp, (void*)gr, (void*)ls}) dfree(c, q);
    HIPCHK(c, e);
    if (loss) {
        double t = 0.0;
        for (float v : hl) t += v;
        *loss = t;
    }
    return M2M_OK;
}

extern "C" m2m_status m2m_mlp_loss_grad_noalloc(m2m_ctx* c, const float* theta, const float* samples, int32_t n,
                                                float* grad, double* loss) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (c->prior.kind != M2M_PRIOR_MLP) return fail(c, M2M_ERR_INVALID, "the context has no learned prior");
    if (!theta || !samples || !grad) return fail(c, M2M_ERR_INVALID, "null argument");
    if (n < kMlpSamples || n % kMlpSamples) return fail(c, M2M_ERR_INVALID, "n must be a positive multiple of 32");
    if (n > kMlpNoAllocMax)
        return fail(c, M2M_ERR_INVALID, "n must be at most " + std::to_string(kMlpNoAllocMax) +
                                            " samples (the size of the static scratch)");
    if (((uintptr_t)samples & 15) != 0) return fail(c, M2M_ERR_INVALID, "samples must be 16-byte aligned");
    if (m2m_status s = sticky(c)) return s;
    if (!c->noalloc_scratch) return fail(c, M2M_ERR_DEVICE, c->noalloc_error);
    MlpArgs a{};
    fill_mlp_args(c, a, c->step);
    a.theta = const_cast<float*>(theta);
    a.sub = reinterpret_cast<float4*>(const_cast<float*>(samples));
    a.batch = n;
    HIPCHK(c, launch_mlp_grad_noalloc(a, c->noalloc_scratch, grad, loss, c->stream));
    return M2M_OK;
}

// ------------------------------------------------------------- launch shape
extern "C" m2m_status m2m_get_launch(const m2m_ctx* c, m2m_launch* out) {
    if (!c || !out) return M2M_ERR_INVALID;
    *out = c->launch;
    return M2M_OK;
}

static m2m_status apply_launch(m2m_ctx* c, const m2m_launch& L) {
    const int tmax = c->prec == M2M_F64 ? 256 : 1024;
    if (L.threads < 64 || L.threads > tmax || L.threads % 64 || (L.ilp != 1 && L.ilp != 2) ||
        L.blocks_per_cu < 1 || L.blocks_per_cu > 64 || L.graph_steps < 0 || L.graph_steps > 100000)
        return fail(c, M2M_ERR_INVALID, "launch shape out of range");
    const bool replan = L.threads != c->plan.threads || L.ilp != c->plan.ilp || L.blocks_per_cu != c->plan.bpc;
    const m2m_launch prev = c->launch;
    c->launch = L;
    if (replan) {
        m2m_status s = make_plan(c, L.threads, L.ilp, L.blocks_per_cu);
        if (s) {
            // keep the context usable: go back to the previous shape
            const std::string why = c->msg;
            c->launch = prev;
            if (make_plan(c, prev.threads, prev.ilp, prev.blocks_per_cu) != M2M_OK) return s;
            c->msg = why;
        }
        return s;
    }
    for (int k = 0; k < 2; ++k)
        if (c->graph[k]) { (void)hipGraphExecDestroy(c->graph[k]); c->graph[k] = nullptr; }
    return M2M_OK;
}

extern "C" m2m_status m2m_set_launch(m2m_ctx* c, const m2m_launch* in) {
    if (!c || !in) return fail(c, M2M_ERR_INVALID, "null argument");
    if (m2m_status s = sticky(c)) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return apply_launch(c, *in);
}

extern "C" m2m_status m2m_kernel_time(const m2m_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return M2M_ERR_INVALID;
    *ms = c->last_kernel_ms;
    *launches = c->last_launches;
    return M2M_OK;
}

// ---------------------------------------------------------------- autotune
namespace {
struct Snapshot {
    std::vector<std::pair<void*, void*>> bufs;   // (live, copy)
    std::vector<size_t> sizes;
};
}  // namespace

static m2m_status snapshot(m2m_ctx* c, Snapshot& s, bool restore) {
    const size_t ts = tsize(c);
    const size_t MJ = (size_t)c->M * c->J, MC = (size_t)c->M * std::max(1, c->NC);
    struct Item { void* p; size_t n; };
    std::vector<Item> items = {{c->state[c->step & 1], state_bytes(c)},
                               {c->ys, MJ * 8}, {c->y, MJ * 8}, {c->delta, MJ * 8}, {c->cvec, MJ * ts},
                               {c->cellmean, MC * ts}, {c->cellmean64, MC * 8}, {c->chunk_chi, 4 * (size_t)c->nchunk * 8},
                               {c->ring, sizeof(StatRow) * (size_t)c->M * kRing}, {c->d_step, 16}};
    if (c->what) items.push_back({c->what, (size_t)c->stride * ts});
    if (c->trc_n) {
        items.push_back({c->trc_Ls, (size_t)c->trc_n * 8});
        items.push_back({c->trc_Ms, (size_t)c->trc_nb * 8});
        items.push_back({c->trc_cL, (size_t)c->trc_n * ts});
        items.push_back({c->trc_cM, (size_t)c->trc_nb * ts});
        items.push_back({c->trc_ll, 8});
    }
    if (c->mlp_theta) {
        items.push_back({c->mlp_theta, sizeof(float) * kMlpNP});
        items.push_back({c->mlp_m, sizeof(float) * kMlpNP});
        items.push_back({c->mlp_v, sizeof(float) * kMlpNP});
        items.push_back({c->mlp_stats, sizeof(double) * 8});
    }
    if (c->mp) {
        const size_t nn = c->mp_pot.nnode, nlm = (size_t)(c->mp_pot.lmax + 1) * (c->mp_pot.lmax + 1);
        items.push_back({c->mp_tab, nn * (ts == 4 ? kMpRowF : kMpW) * ts});
        items.push_back({c->mp_A64, nn * nlm * 8});
        items.push_back({c->mp_B64, nn * nlm * 8});
        items.push_back({c->mp_acc[c->step & 1], 3 * (size_t)c->stride * ts});
    }
    if (!restore) {
        for (auto& it : items) {
            void* cp = nullptr;
            if (hipMalloc(&cp, it.n) != hipSuccess) {
                (void)hipGetLastError();
                for (auto& b : s.bufs) (void)hipFree(b.second);
                s.bufs.clear();
                return fail(c, M2M_ERR_NOMEM, "autotune snapshot allocation failed");
            }
            HIPCHK(c, hipMemcpy(cp, it.p, it.n, hipMemcpyDeviceToDevice));
            s.bufs.push_back({it.p, cp});
            s.sizes.push_back(it.n);
        }
    } else {
        for (size_t k = 0; k < s.bufs.size(); ++k)
            HIPCHK(c, hipMemcpy(s.bufs[k].first, s.bufs[k].second, s.sizes[k], hipMemcpyDeviceToDevice));
        HIPCHK(c, hipMemset(c->flag, 0, sizeof(int)));
    }
    return M2M_OK;
}

static std::string tune_key(const m2m_ctx* c) {
    char buf[256];
    snprintf(buf, sizeof buf, "gfx950|p%d|k%d|N%lld|M%d|J%d|C%d|P%d", c->prec, c->pot_kind, (long long)c->N, c->M, c->J,
             c->NC, c->prior.kind);
    return buf;
}

static bool cache_lookup(const std::string& key, m2m_launch* L) {
    const char* path = std::getenv("M2M_AUTOTUNE_CACHE");
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        // one JSON object per line: {"key": "...", "threads": T, "ilp": I, "blocks_per_cu": B}
        char k[256];
        int t, i, b;
        if (std::sscanf(line, " {\"key\": \"%255[^\"]\", \"threads\": %d, \"ilp\": %d, \"blocks_per_cu\": %d", k, &t, &i, &b) == 4 &&
            key == k) {
            L->threads = t;
            L->ilp = i;
            L->blocks_per_cu = b;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void cache_store(const std::string& key, const m2m_launch& L) {
    const char* path = std::getenv("M2M_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"threads\": %d, \"ilp\": %d, \"blocks_per_cu\": %d}\n", key.c_str(), L.threads, L.ilp,
                 L.blocks_per_cu);
    std::fclose(f);
}

extern "C" m2m_status m2m_autotune(m2m_ctx* c, int32_t trial_steps, m2m_launch* chosen) {
    if (!c) return fail(nullptr, M2M_ERR_INVALID, "ctx is NULL");
    if (m2m_status s = sticky(c)) return s;
    if (trial_steps < 1) return fail(c, M2M_ERR_INVALID, "trial_steps must be >= 1");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const m2m_launch keep = c->launch;
    m2m_launch best = keep;
    const std::string key = tune_key(c);
    if (!cache_lookup(key, &best)) {
        Snapshot snap;
        if (m2m_status s = snapshot(c, snap, false)) return s;
        const int64_t step0 = c->step, mlp_t0 = c->mlp_t;
        double best_ms = INFINITY;
        std::vector<int> threads = c->prec == M2M_F64 ? std::vector<int>{64, 128, 256} : std::vector<int>{256, 512, 1024};
        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        m2m_status err = M2M_OK;
        for (int t : threads)
            for (int ilp : {1, 2})
                for (int bpc : {1, 2, 4}) {
                    m2m_launch L = keep;
                    L.threads = t;
                    L.ilp = ilp;
                    L.blocks_per_cu = bpc;
                    L.graph_steps = 0;
                    L.timing = 0;
                    if ((err = apply_launch(c, L))) {
                        if (err == M2M_ERR_UNSUPPORTED) { err = M2M_OK; continue; }
                        goto done;
                    }
                    (void)launch_one(c, c->step);   // warm-up
                    ++c->step;
                    if (hipEventRecord(e0, c->stream) != hipSuccess) { err = fail(c, M2M_ERR_DEVICE, "event"); goto done; }
                    for (int k = 0; k < trial_steps; ++k) { (void)launch_one(c, c->step); ++c->step; }
                    (void)hipEventRecord(e1, c->stream);
                    (void)hipEventSynchronize(e1);
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    int flag = 0;
                    (void)hipMemcpy(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost);
                    if (!flag && ms < best_ms) { best_ms = ms; best = L; }
                    if ((err = snapshot(c, snap, true))) goto done;
                    c->step = step0;
                    c->mlp_t = mlp_t0;
                }
    done:
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        for (auto& b : snap.bufs) (void)hipFree(b.second);
        c->step = step0;
        c->mlp_t = mlp_t0;
        if (err) return err;
        cache_store(key, best);
    }
    best.graph_steps = keep.graph_steps;
    best.timing = keep.timing;
    if (m2m_status s = apply_launch(c, best)) return s;
    if (chosen) *chosen = c->launch;
    return M2M_OK;
}

// ------------------------------------------------------------------ destroy
extern "C" void m2m_destroy(m2m_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k)
        if (c->graph[k]) (void)hipGraphExecDestroy(c->graph[k]);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

extern "C" const char* m2m_last_error(const m2m_ctx* c) {
    return c ? c->msg.c_str() : g_create_error.c_str();
}
