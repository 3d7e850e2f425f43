// step.hip -- fused M2M step kernel (plus the energy-range and prior readback
// kernels).
//
// One launch of step_kernel performs, for every particle of every model (the
// per-timestep loop of the made-to-measure method, section 2 of the paper):
//   the weight update with the current deviations and priors (maximising
//   F = -chi^2/2 + mu S, eq. 1 and 2), the kick-drift-kick push in the analytic
//   potential, and the scatter of w * K_j of the new state into LDS-privatised
//   observable histograms, plus the moving-prior cell sums (section 2.1).
// The bins and the prior cell of a particle are decided once, for the new
// state, and stored as 16-bit tags beside the state: the next step's update
// reads them instead of deciding again.
// Each block owns a contiguous range of tiles; a tile never straddles models.
// When a block moves to another model (batched form) or finishes, it writes
// its LDS histograms to its own partial slot (no atomics, deterministic
// placement); finalize.hip sums the slots.
#include <hip/hip_ext.h>

#include "particle.h"

namespace m2m {

// One particle's step: update the weight with the bins and cell of the current
// state (its tags), push, decide the bins and cell of the new state, store, and
// scatter into the histograms.  With kObserve the particle is neither updated
// nor moved: its current bins and cell are decided and stored.
// FP32 kernels decide in FP32; a decision inside its guard band is left open
// and flagged in the returned mask (bit b: binning b, bits NB..NB+2: the cell's
// axes), to be re-taken in FP64 by fix_one() from the stored new state; FP64
// kernels decide in FP64 and return 0.

template <int POT, int NB, uint64_t SIG, int CAX, typename T, typename PT>
__device__ __forceinline__ unsigned particle_step(const StepArgs<T, PT>& a, const Blk<T>& B, Acc& acc, int64_t p,
                                                  T x, T y, T z, T vx, T vy, T vz, T w, T what_p,
                                                  const uint16_t (&tg)[kMaxBin + 1], uint32_t fl, uint32_t rb) {
    // fl: the step flags; rb: bytes per value row
    const Layout<T>& L = a.lay;
    const LayoutView<SIG, T> V{L};
    const uint32_t o = uint32_t(p) * uint32_t(sizeof(T));
    const uint32_t ot = 7 * rb + uint32_t(p) * 2u;                 // tag of row 0

    const int nbin = V.nbin();
    T wn = w, phi = T(0);
    bool have_phi = false;
    if (!(fl & kObserve)) {
        wn = weight_update<NB, SIG, 0>(a, B, acc, p, vy, vz, w, what_p, tg, fl, a.jpad);
        if (!(fl & kFrozen)) {
            // kick-drift-kick
            T ax, ay, az;
            potential<POT, T>(B.pot, x, y, z, phi, ax, ay, az);
            const T hdt = T(0.5) * a.dt;
            vx += hdt * ax; vy += hdt * ay; vz += hdt * az;
            x += a.dt * vx; y += a.dt * vy; z += a.dt * vz;
            potential<POT, T>(B.pot, x, y, z, phi, ax, ay, az);
            vx += hdt * ax; vy += hdt * ay; vz += hdt * az;
            have_phi = true;
        }
        st_at(a.out, o, x);
        st_at(a.out, o + rb, y);
        st_at(a.out, o + 2 * rb, z);
        st_at(a.out, o + 3 * rb, vx);
        st_at(a.out, o + 4 * rb, vy);
        st_at(a.out, o + 5 * rb, vz);
        st_at(a.out, o + 6 * rb, wn);
    }
    // bins and cell of the new state
    unsigned open = 0;
    const T vl = line_of_sight(vy, vz, L.sini, L.cosi);
    const float yc = float(y * L.cosi), zs = float(z * L.sini);
    const float Ys = yc - zs, aYs = fabsf(yc) + fabsf(zs);
    // (no branches: a decision left open stores a provisional tag, which the
    // fix-up overwrites, and scatters to the lane's trash slot, as does a
    // particle outside the binning)
    const int lane = threadIdx.x & 63;
    #pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nbin) break;
        int k;
        bool take;
        if constexpr (sizeof(T) == 4) {
            bool sure;
            k = bin_fast(L.b[b], V.kind(b), B.ed, x, y, z, Ys, aYs, sure);
            open |= sure ? 0u : 1u << b;
            take = sure && k >= 0;
        } else {
            const Exact* ex = a.ex;
            const BinDesc<T>& d = L.b[b];
            k = bin_f64(V.kind(b), ex->cosd, ex->sind, ex->x0d[b], ex->wxd[b], d.nx, ex->y0d[b], ex->wyd[b], d.ny,
                        B.ed64 + d.edge0, d.nb + 1, x, y, z);
            take = k >= 0;
        }
        st_at<uint16_t>(a.out, ot + b * (rb / uint32_t(sizeof(T)) * 2u), k < 0 ? kNoBin : (uint16_t)k);
        scatter_bin(V, B.hist, b, k, take, a.jpad + lane, wn, vl, B.gh);
    }
    int cell = 0;
    if (fl & kAccum) {
        if (!have_phi) {
            T ax, ay, az;
            potential<POT, T>(B.pot, x, y, z, phi, ax, ay, az);
        }
        unsigned am = 0;
        if constexpr (sizeof(T) == 4) {
            const float KE = 0.5f * (vx * vx + vy * vy + vz * vz);
            am = cell_fast<POT, CAX>(B.pot, B.et, a.cells, B.Emin, B.sE, B.cg, KE, phi, x, y, z, vx, vy, vz, cell);
            open |= am << NB;
        } else {
            cell = prior_cell_f64<POT>(B.pot, B.lct, a.cells, a.ex->erange[2 * B.m], a.ex->erange[2 * B.m + 1], x, y, z,
                                       vx, vy, vz);
        }
        st_at<uint16_t>(a.out, ot + a.cellrow * (rb / uint32_t(sizeof(T)) * 2u), (uint16_t)cell);
        const int ci = am == 0 ? cell : a.cells.ncell + lane;
        atomicAdd(&B.csum[ci], double(wn));
        atomicAdd(&B.ccnt[ci], 1u);
    }
    return open;
}

// The decisions particle_step left open for particle p (mask `open`), taken in
// FP64 from the FP32 coordinates of its new state, read back from the output
// buffer where this wave stored them (with the provisional FP32 cell tag, exact
// on the axes not left open), then stored and scattered.  Only the open axes of
// the cell are re-taken: E needs one FP64 potential, L/Lc or Lz/Lc the
// circular-orbit Lc(E) as well, Lz/L neither.
// Out of line (its FP64 working set would otherwise raise the register use of
// the whole kernel), with address-space-qualified pointers so that neither side
// falls back to flat addressing; called from the queue drain only.
using cExact = const __attribute__((address_space(4))) Exact;
using gF32 = __attribute__((address_space(1))) float;
using lF64 = __attribute__((address_space(3))) double;
using lU32 = __attribute__((address_space(3))) unsigned;
template <int POT, int NB>
__device__ __noinline__ void fix_one(cExact* ex, int m, unsigned open, int64_t p, int64_t stride, int cellrow,
                                     gF32* out, lF64* hist, lF64* csum, lU32* ccnt, float lcE0, float lcEinv, float sini,
                                     float cosi) {
    const float x = out[p], y = out[stride + p], z = out[2 * stride + p];
    const float vx = out[3 * stride + p], vy = out[4 * stride + p], vz = out[5 * stride + p];
    const float wn = out[6 * stride + p];
    __attribute__((address_space(1))) uint16_t* tags =
        reinterpret_cast<__attribute__((address_space(1))) uint16_t*>(out + 7 * stride);
    const float vl = line_of_sight(vy, vz, sini, cosi);
    #pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (!(open & (1u << b))) continue;
        const int kind = ex->lay.b[b].kind, nx = ex->lay.b[b].nx, ny = ex->lay.b[b].ny, nb = ex->lay.b[b].nb;
        const int k = bin_f64(kind, ex->cosd, ex->sind, ex->x0d[b], ex->wxd[b], nx, ex->y0d[b], ex->wyd[b], ny,
                              ex->edges + ex->lay.b[b].edge0, nb + 1, double(x), double(y), double(z));
        tags[b * stride + p] = k < 0 ? kNoBin : (uint16_t)k;
        if (k < 0) continue;
        const int base = ex->lay.b[b].off + k, mom = ex->lay.b[b].mom;
        const float* gv = ex->gh + 2 * (ex->lay.b[b].gh0 + k);
        for (int mm = 0; mm < ex->lay.b[b].nmom; ++mm)
            __hip_atomic_fetch_add(&hist[base + mm * nb],
                                   double(wn * kernel_value<float>((mom >> (kMomBits * mm)) & 7, vl, gv)),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    const unsigned am = (open >> NB) & 7u;
    if (am) {
        Cells cells;
        cells.n0 = ex->cells.n0;
        cells.n1 = ex->cells.n1;
        cells.n2 = ex->cells.n2;
        cells.ax2 = ex->cells.ax2;
        cells.ncell = ex->cells.ncell;
        const int n1 = cells.n1, n2 = cells.n2;
        const int cell = tags[cellrow * stride + p];
        int iE = cell / (n1 * n2), i2 = (cell / n2) % n1, i3 = cell % n2;
        const double X = x, Y = y, Z = z, VX = vx, VY = vy, VZ = vz;
        if (am & 3u) {
            const Pot<double> pd = ex->pots[m];
            const double E = energy64<POT>(pd, X, Y, Z, VX, VY, VZ);
            if (am & 1u) iE = cell_axis_E(cells, ex->erange[2 * m], ex->erange[2 * m + 1], E);
            if (am & 2u) {
                double L, Lz;
                angmom64(X, Y, Z, VX, VY, VZ, L, Lz);
                const double Lc = lc_seeded<POT>(pd, ex->lctab + pd.lc_off, ex->rce + (size_t)m * kLcE,
                                                 double(lcE0), double(lcEinv), E);
                i2 = cell_axis_2(cells, L, Lz, Lc);
            }
        }
        if (am & 4u) {
            double L, Lz;
            angmom64(X, Y, Z, VX, VY, VZ, L, Lz);
            i3 = cell_axis_3(cells, L, Lz);
        }
        const int c = (iE * n1 + i2) * n2 + i3;
        tags[cellrow * stride + p] = (uint16_t)c;
        __hip_atomic_fetch_add(&csum[c], double(wn), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&ccnt[c], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// MODE: the step flags at run time (0), or compiled in: a stepping kernel of a
// histogram prior refreshed every step with the exponential law (1), an
// observe-only pass that takes the prior cells (2), a stepping kernel with
// stored per-particle priors and no cells (3: the learned prior between
// refreshes, a periodic prior's steps that take no cells), or mode 1 with the
// discrete tracers' term of G (4).
constexpr uint32_t kHotFlags = kExpLaw | (1u << kWhatShift) | kAccum;
constexpr uint32_t kObsCells = kObserve | kAccum;
constexpr uint32_t kHotStored = kExpLaw | (3u << kWhatShift);
constexpr uint32_t kHotTracers = kHotFlags | kTracers;

template <typename T, typename PT, int POT, int NB, uint64_t SIG, int CAX, int MODE, int ILP>
__global__ void __launch_bounds__(sizeof(T) == 8 ? 256 : 1024) step_kernel(StepArgs<T, PT> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    warm_kernargs<sizeof(StepArgs<T, PT>)>();
    // an earlier step failed: the whole step is a no-op (the flag, as it stood
    // when the kernel started, is read through the scalar cache and checked
    // after the first model's tables are in LDS and before the first store, so
    // that no load of the prologue waits for it)
    const int failed = ro(a.flag, 0);
    // the block's start in one load; everything the prologue loads next (model
    // tables, the update table, cell means, the first tile's particles) depends
    // on it alone
    const BlockDesc bd = ro(a.block_desc, blockIdx.x);

    constexpr bool F32 = sizeof(T) == 4;
    const int J = a.lay.J, NC = a.cells.ncell, JP = a.jpad, NE = (a.nedge + 1) & ~1;
    const int nt = blockDim.x, tid = threadIdx.x;
    double* hist = reinterpret_cast<double*>(smem);                 // J (padded to JP), then kTrash
    double* csum = hist + JP + kTrash;                               // NC, then kTrash
    double* ed64 = csum + NC + kTrash;                               // edges, FP64
    unsigned* ctr = reinterpret_cast<unsigned*>(ed64 + NE);         // work counter (2 doubles' room)
    double* wst = ed64 + NE + 2;                                     // 4 per wave: weight statistics
    unsigned* ccnt = reinterpret_cast<unsigned*>(wst + 64);          // NC (padded to even), then kTrash
    T* cl = reinterpret_cast<T*>(ccnt + ((NC + 1) & ~1) + kTrash);   // J : Dt_j / sigma_j, zero to JP + 2
    T* cm = cl + JP + 2;                                             // NC: cell means
    T* ed = cm + ((NC + 1) & ~1);                                    // edges in T
    T* lct = ed + NE;                                                // circular-orbit energies (FP64)
    float2* etl = reinterpret_cast<float2*>(lct + kLcTab);           // uniform-E Lc table (FP32, with cells)
    uint2* fq = reinterpret_cast<uint2*>(etl + (F32 && NC ? kLcE : 0));  // per wave: kFixQ open decisions (FP32)
    T* ghl = reinterpret_cast<T*>(fq + (F32 ? kFixQ * (blockDim.x >> 6) : 0));   // Gauss-Hermite (V, 1/sigma) pairs

    for (int i = tid; i < a.nedge; i += nt) { ed[i] = a.edges[i]; ed64[i] = a.edges64[i]; }
    for (int i = tid; i < 2 * a.lay.ngh; i += nt) ghl[i] = a.ghtab[i];

    const uint32_t fl = MODE == 1   ? kHotFlags
                        : MODE == 2 ? kObsCells
                        : MODE == 3 ? kHotStored
                        : MODE == 4 ? kHotTracers
                                    : a.flags;
    const uint32_t wm = (fl >> kWhatShift) & 3u;
    const bool want_cm = wm == 1 || wm == 2;
    const bool accum = fl & kAccum;
    const bool stepping = !(fl & kObserve);
    Blk<T> B;
    B.hist = hist; B.csum = csum; B.ccnt = ccnt; B.cl = cl; B.cm = cm; B.ed = ed; B.ed64 = ed64;
    B.lct = lct;
    B.gh = ghl;
    Acc acc;

    // Work is handed out per wave in chunks of CH = 64 ILP particles of the
    // current segment (the block's run of tiles of one model): wave w starts
    // with chunk w and then takes the next unclaimed chunk from a counter in
    // LDS, so that waves slowed by a fix-up or by the issue order simply take
    // fewer chunks and the block's waves finish together.  The next chunk's
    // particles are loaded while the current one is processed.
    constexpr int CH = 64 * ILP;
    const int nw = nt >> 6, wid = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    struct Regs {
        T x[ILP], y[ILP], z[ILP], vx[ILP], vy[ILP], vz[ILP], w[ILP], wh[ILP];
        uint16_t tg[ILP][kMaxBin + 1];
    };
    // the particles of chunk c of the segment [P0, P0 + n) (values and the tags
    // of the current state)
    auto load_chunk = [&](int64_t P0, int n, int c, Regs& R) {
        const uint32_t rb = opaque(uint32_t(a.stride * sizeof(T))), tr = uint32_t(a.stride * 2);
        #pragma unroll
        for (int k = 0; k < ILP; ++k) {
            const int i = c * CH + k * 64 + lane;
            if (i < n) {
                const int64_t p = P0 + i;
                const uint32_t o = uint32_t(p) * uint32_t(sizeof(T)), ot = 7 * rb + uint32_t(p) * 2u;
                R.x[k] = ld_at<T>(a.in, o);
                R.y[k] = ld_at<T>(a.in, o + rb);
                R.z[k] = ld_at<T>(a.in, o + 2 * rb);
                R.vx[k] = ld_at<T>(a.in, o + 3 * rb);
                R.vy[k] = ld_at<T>(a.in, o + 4 * rb);
                R.vz[k] = ld_at<T>(a.in, o + 5 * rb);
                R.w[k] = ld_at<T>(a.in, o + 6 * rb);
                #pragma unroll
                for (int b = 0; b < kMaxBin; ++b)
                    R.tg[k][b] = (stepping && b < NB && b < LayoutView<SIG, T>{a.lay}.nbin())
                                     ? ld_at<uint16_t>(a.in, ot + b * tr) : kNoBin;
                R.tg[k][kMaxBin] = (stepping && want_cm) ? ld_at<uint16_t>(a.in, ot + a.cellrow * tr) : 0;
                R.wh[k] = (stepping && wm == 3) ? a.what[p] : T(1);
            }
        }
    };
    // two register sets, used in turn: the chunk being processed and the next
    // one being loaded (no copy between them)
    Regs R0;
    // the first segment (its first chunk's loads go out before the tables')
    int m = bd.m0, n = bd.n0, slot = bd.slot0, te = bd.tseg1;
    int64_t P0 = bd.p0;
    int ts = bd.t0;
    if (ts < bd.t1 && wid * CH < n) load_chunk(P0, n, wid, R0);
    // FP32: the decisions this wave left open, (particle, mask) pairs queued in
    // LDS and re-taken in FP64 all lanes at a time when the queue fills up or the
    // segment ends (qn is wave-uniform)
    uint2* myq = fq + wid * kFixQ;
    int qn = 0;

    while (ts < bd.t1) {
        // the segment's model: tables, histograms and the work counter
        B.m = m;
        B.pot = ro(a.pots, m);
        B.Emin = ro(a.erange, 2 * m);
        B.sE = T(a.cells.n0) / (ro(a.erange, 2 * m + 1) - ro(a.erange, 2 * m));
        if constexpr (F32) B.cg = cell_guard(B.Emin, ro(a.erange, 2 * m + 1), B.sE);
        B.wflat = ro(a.flatw, m);
        for (int j = tid; j < J; j += nt) { hist[j] = 0.0; cl[j] = a.cvec[(size_t)m * J + j]; }
        if (tid < JP + 2 - J) cl[J + tid] = T(0);   // the entries bins without a particle read
        if (accum) for (int c = tid; c < NC; c += nt) { csum[c] = 0.0; ccnt[c] = 0u; }
        if (want_cm) for (int c = tid; c < NC; c += nt) cm[c] = a.cellmean[(size_t)m * NC + c];
        if (NC && !F32) for (int i = tid; i < kLcTab; i += nt) lct[i] = a.lctab[(size_t)B.pot.lc_off + i];
        if (F32 && accum) {
            // the model's uniform-E Lc table into LDS (a global gather in the
            // particle loop would wait behind the chunk's stores and the next
            // chunk's loads)
            const float4* src = reinterpret_cast<const float4*>(a.lcetab + 2 * (size_t)m * kLcE);
            for (int i = tid; i < kLcE / 2; i += nt) {
                const float4 v = src[i];
                etl[2 * i] = make_float2(v.x, v.y);
                etl[2 * i + 1] = make_float2(v.z, v.w);
            }
        }
        if (tid == 0) *ctr = 0u;
        B.et = etl;
        __syncthreads();
        if (failed) return;   // (uniform: every thread leaves here, before any store)

        const int nch = (n + CH - 1) / CH;
        int c = wid;
        while (true) {
            if constexpr (F32) {
                // re-take the queued open decisions when another chunk might not
                // fit, and at the end of the segment (before the next chunk's loads
                // are issued, so that waiting for those never waits on these)
                if (qn > kFixQ - CH || (c >= nch && qn > 0)) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");   // this wave's stores are complete
                    for (int i = lane; i < qn; i += 64) {
                        const uint2 e = myq[i];
                        fix_one<POT, NB>((cExact*)a.ex, B.m, e.y, (int64_t)e.x, a.stride, a.cellrow, (gF32*)a.out,
                                         (lF64*)hist, (lF64*)csum, (lU32*)ccnt, B.pot.lcE0, B.pot.lcEinv, a.lay.sini,
                                         a.lay.cosi);
                    }
                    qn = 0;
                }
            }
            if (c >= nch) break;
            // this chunk's particles (loaded one chunk ago), then the next chunk's loads
            const Regs cur_r = R0;
            unsigned got = 0;
            if (lane == 0) got = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int cn = nw + (int)__builtin_amdgcn_readfirstlane(got);
            if (cn < nch) load_chunk(P0, n, cn, R0);
            const uint32_t flo = MODE ? fl : opaque(a.flags), rbo = opaque(uint32_t(a.stride * sizeof(T)));
            #pragma unroll
            for (int k = 0; k < ILP; ++k) {
                const int i = c * CH + k * 64 + lane;
                const unsigned o = i < n ? particle_step<POT, NB, SIG, CAX>(a, B, acc, P0 + i, cur_r.x[k], cur_r.y[k],
                                                                           cur_r.z[k], cur_r.vx[k], cur_r.vy[k],
                                                                           cur_r.vz[k], cur_r.w[k], cur_r.wh[k],
                                                                           cur_r.tg[k], flo, rbo)
                                         : 0u;
                if constexpr (F32) {
                    // queue the open decisions of this 64-particle group
                    const unsigned long long bm = __ballot(o != 0u);
                    if (bm) {
                        const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi(
                                                 uint32_t(bm >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bm), 0u));
                        if (o) myq[pos] = make_uint2(uint32_t(P0 + i), o);
                        qn += __popcll(bm);
                    }
                }
            }
            c = cn;
        }

        // flush the segment's histograms to its partial slot, and its weight
        // statistics (observing only, they belong to the kernel that updated
        // the weights)
        if (stepping) wave_stats(acc.S, acc.W, acc.W2, acc.mn, wst);
        __syncthreads();
        if (stepping && tid == 0) block_stats_write(wst, nw, a.seg_stats + 4 * (size_t)slot);
        PT* dst = a.part + ro(a.slot_base, slot);
        const int64_t cs = ro(a.slot_stride, slot);
        auto at = [&](int j) -> PT& { return dst[(j / kFinCols) * cs + j % kFinCols]; };
        for (int j = tid; j < J; j += nt) at(j) = PT(hist[j]);
        if (accum)
            for (int c2 = tid; c2 < NC; c2 += nt) { at(JP + 2 * c2) = PT(csum[c2]); at(JP + 2 * c2 + 1) = PT(ccnt[c2]); }
        acc.S = acc.W = acc.W2 = 0;
        acc.mn = INFINITY;

        // the next segment, if any (a block spanning models)
        ts = te;
        if (ts >= bd.t1) break;
        m = ro(a.tile_model, ts);
        P0 = ro(a.tile_p0, ts);
        te = ts;
        while (te < bd.t1 && ro(a.tile_model, te) == m) ++te;
        n = (int)(ro(a.tile_p0, te - 1) + ro(a.tile_cnt, te - 1) - P0);
        ++slot;
        __syncthreads();   // every thread has read the LDS of the flushed segment
        if (wid * CH < n) load_chunk(P0, n, wid, R0);
    }
    if (acc.bad) {
        __hip_atomic_fetch_or(a.flag, (int)acc.bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *a.bad_step = *a.d_step;
    }
}

// ---------------------------------------------------- energy range (at create)
// Min and max of E(0) over each model's particles, in FP64 from the stored
// values (the range the prior's energy axis spans when the caller gives none).
template <typename T, int POT>
__global__ void __launch_bounds__(256) erange_kernel(ErangeArgs<T> a) {
    __shared__ double rmin[4], rmax[4];
    const int t0 = a.block_tile0[blockIdx.x], t1 = a.block_tile0[blockIdx.x + 1];
    int slot = a.block_slot0[blockIdx.x] - 1, cur = -1;
    double lo = INFINITY, hi = -INFINITY;
    Pot<double> pot;
    for (int t = t0; t <= t1; ++t) {
        const int m = t < t1 ? a.tile_model[t] : -2;
        if (m != cur) {
            if (cur >= 0) {
                lo = wave_min(lo);
                hi = -wave_min(-hi);
                if ((threadIdx.x & 63) == 0) { rmin[threadIdx.x >> 6] = lo; rmax[threadIdx.x >> 6] = hi; }
                __syncthreads();
                if (threadIdx.x == 0) {
                    double l = rmin[0], h = rmax[0];
                    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) { l = fmin(l, rmin[i]); h = fmax(h, rmax[i]); }
                    a.out[2 * slot] = l;
                    a.out[2 * slot + 1] = h;
                }
                __syncthreads();
                lo = INFINITY; hi = -INFINITY;
            }
            if (m < 0) break;
            cur = m;
            ++slot;
            pot = a.pots[m];
        }
        const int64_t p0 = a.tile_p0[t];
        const int cnt = a.tile_cnt[t];
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int64_t p = p0 + i;
            T x = a.in[p], y = a.in[a.stride + p], z = a.in[2 * a.stride + p];
            T vx = a.in[3 * a.stride + p], vy = a.in[4 * a.stride + p], vz = a.in[5 * a.stride + p];
            double phi, ax, ay, az;
            potential<POT, double>(pot, double(x), double(y), double(z), phi, ax, ay, az);
            const double E = 0.5 * (double(vx) * vx + double(vy) * vy + double(vz) * vz) + phi;
            lo = fmin(lo, E);
            hi = fmax(hi, E);
        }
    }
}

// ------------------------------------------ priors of the current state (readback)
// The prior cell of every particle is its stored tag (decided when the state
// was made).
template <typename T>
__global__ void __launch_bounds__(256) gather_kernel(GatherArgs<T> a) {
    const int t0 = a.block_tile0[blockIdx.x], t1 = a.block_tile0[blockIdx.x + 1];
    for (int t = t0; t < t1; ++t) {
        const int m = a.tile_model[t];
        const int64_t p0 = a.tile_p0[t];
        const int cnt = a.tile_cnt[t];
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int64_t p = p0 + i;
            T wh;
            if (a.what_mode == 0) wh = a.flatw[m];
            else if (a.what_mode == 3) wh = a.what[p];
            else wh = a.cellmean[(size_t)m * a.cells.ncell + a.tin[a.cellrow * a.stride + p]];
            a.out[p] = wh;
        }
    }
}

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_gather(const GatherArgs<T>& a, int pot_kind, int blocks, hipStream_t s) {
    (void)pot_kind;
    hipLaunchKernelGGL((gather_kernel<T>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_gather<float>(const GatherArgs<float>&, int, int, hipStream_t);
template hipError_t launch_gather<double>(const GatherArgs<double>&, int, int, hipStream_t);

template <typename T, typename PT, int POT, int NB, uint64_t SIG, int CAX, int MODE>
static hipError_t launch_k(const StepArgs<T, PT>& a, int ilp, int blocks, int threads, size_t lds, hipStream_t s,
                           hipEvent_t e0, hipEvent_t e1) {
    if (e0 || e1) {
        // (timing: the events take the kernel's own start and end times)
        if (ilp == 1)
            hipExtLaunchKernelGGL((step_kernel<T, PT, POT, NB, SIG, CAX, MODE, 1>), dim3(blocks), dim3(threads),
                                  (uint32_t)lds, s, e0, e1, 0u, a);
        else
            hipExtLaunchKernelGGL((step_kernel<T, PT, POT, NB, SIG, CAX, MODE, 2>), dim3(blocks), dim3(threads),
                                  (uint32_t)lds, s, e0, e1, 0u, a);
    } else if (ilp == 1) {
        hipLaunchKernelGGL((step_kernel<T, PT, POT, NB, SIG, CAX, MODE, 1>), dim3(blocks), dim3(threads), lds, s, a);
    } else {
        hipLaunchKernelGGL((step_kernel<T, PT, POT, NB, SIG, CAX, MODE, 2>), dim3(blocks), dim3(threads), lds, s, a);
    }
    return hipGetLastError();
}

// A signature kernel with the prior's cell axes and the step's flags compiled in
// when they are the common ones (CAX1; the stepping or observing flags of a
// histogram prior refreshed every step), else with both at run time.
template <typename T, typename PT, int POT, int NB, uint64_t SIG, int CAX1>
static hipError_t launch_cax(const StepArgs<T, PT>& a, int ilp, int blocks, int threads, size_t lds, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1) {
    if (a.flags == kHotStored) return launch_k<T, PT, POT, NB, SIG, kCaxRuntime, 3>(a, ilp, blocks, threads, lds, s, e0, e1);
    if (a.cells.ncell > 0 && cax_of(a.cells) == CAX1) {
        if (a.flags == kHotFlags) return launch_k<T, PT, POT, NB, SIG, CAX1, 1>(a, ilp, blocks, threads, lds, s, e0, e1);
        if (a.flags == kHotTracers) return launch_k<T, PT, POT, NB, SIG, CAX1, 4>(a, ilp, blocks, threads, lds, s, e0, e1);
        if ((a.flags & ~(3u << kWhatShift)) == kObsCells)
            return launch_k<T, PT, POT, NB, SIG, CAX1, 2>(a, ilp, blocks, threads, lds, s, e0, e1);
    }
    return launch_k<T, PT, POT, NB, SIG, kCaxRuntime, 0>(a, ilp, blocks, threads, lds, s, e0, e1);
}

// FP32 layouts with a compiled signature get their own kernels (for the log
// potential's (E, Lz/Lc) priors and the spherical potentials' (E, L/Lc) priors
// with the cell axes compiled in as well); every other layout runs the kernels
// compiled for at most NB = 2 or 4 binnings.
template <typename T, typename PT, int POT>
static hipError_t launch_step_pot(const StepArgs<T, PT>& a, uint64_t sig, int nbin, int ilp, int blocks, int threads,
                                  size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (sizeof(T) == 4 && POT == 1) {
        if (sig == kSigPixKin) return launch_cax<T, PT, POT, 2, kSigPixKin, kCaxLzNo3>(a, ilp, blocks, threads, lds, s, e0, e1);
        if (sig == kSigPixKinShell)
            return launch_cax<T, PT, POT, 4, kSigPixKinShell, kCaxLzNo3>(a, ilp, blocks, threads, lds, s, e0, e1);
    }
    if constexpr (sizeof(T) == 4 && POT != 1)
        if (sig == kSigShellAnn) return launch_cax<T, PT, POT, 2, kSigShellAnn, kCaxLNo3>(a, ilp, blocks, threads, lds, s, e0, e1);
    if (nbin <= 2) return launch_k<T, PT, POT, 2, 0, kCaxRuntime, 0>(a, ilp, blocks, threads, lds, s, e0, e1);
    return launch_k<T, PT, POT, 4, 0, kCaxRuntime, 0>(a, ilp, blocks, threads, lds, s, e0, e1);
}

template <typename T, typename PT>
hipError_t launch_step(const StepArgs<T, PT>& a, int pot_kind, uint64_t sig, int nbin, int ilp, int blocks,
                       int threads, size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (pot_kind) {
        case 0: return launch_step_pot<T, PT, 0>(a, sig, nbin, ilp, blocks, threads, lds, s, e0, e1);
        case 1: return launch_step_pot<T, PT, 1>(a, sig, nbin, ilp, blocks, threads, lds, s, e0, e1);
        default: return launch_step_pot<T, PT, 2>(a, sig, nbin, ilp, blocks, threads, lds, s, e0, e1);
    }
}

template <typename T, typename PT, int POT, int NB, uint64_t SIG, int CAX, int MODE>
static hipError_t set_lds_k(size_t lds) {
    for (const void* f : {(const void*)step_kernel<T, PT, POT, NB, SIG, CAX, MODE, 1>,
                          (const void*)step_kernel<T, PT, POT, NB, SIG, CAX, MODE, 2>}) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, typename PT, int POT, int NB, uint64_t SIG, int CAX1>
static hipError_t set_lds_sig(size_t lds) {
    hipError_t e = set_lds_k<T, PT, POT, NB, SIG, kCaxRuntime, 0>(lds);
    if (e == hipSuccess) e = set_lds_k<T, PT, POT, NB, SIG, CAX1, 1>(lds);
    if (e == hipSuccess) e = set_lds_k<T, PT, POT, NB, SIG, CAX1, 2>(lds);
    if (e == hipSuccess) e = set_lds_k<T, PT, POT, NB, SIG, kCaxRuntime, 3>(lds);
    if (e == hipSuccess) e = set_lds_k<T, PT, POT, NB, SIG, CAX1, 4>(lds);
    return e;
}

template <typename T, typename PT, int POT>
static hipError_t set_lds_pot(size_t lds) {
    hipError_t e = set_lds_k<T, PT, POT, 2, 0, kCaxRuntime, 0>(lds);
    if (e == hipSuccess) e = set_lds_k<T, PT, POT, 4, 0, kCaxRuntime, 0>(lds);
    if constexpr (sizeof(T) == 4 && POT == 1) {
        if (e == hipSuccess) e = set_lds_sig<T, PT, POT, 2, kSigPixKin, kCaxLzNo3>(lds);
        if (e == hipSuccess) e = set_lds_sig<T, PT, POT, 4, kSigPixKinShell, kCaxLzNo3>(lds);
    }
    if constexpr (sizeof(T) == 4 && POT != 1)
        if (e == hipSuccess) e = set_lds_sig<T, PT, POT, 2, kSigShellAnn, kCaxLNo3>(lds);
    return e;
}

template <typename T, typename PT>
hipError_t set_step_lds_limit(int pot_kind, size_t lds) {
    switch (pot_kind) {
        case 0: return set_lds_pot<T, PT, 0>(lds);
        case 1: return set_lds_pot<T, PT, 1>(lds);
        default: return set_lds_pot<T, PT, 2>(lds);
    }
}

template <typename T>
hipError_t launch_erange(const ErangeArgs<T>& a, int pot_kind, int blocks, hipStream_t s) {
    switch (pot_kind) {
        case 0: hipLaunchKernelGGL((erange_kernel<T, 0>), dim3(blocks), dim3(256), 0, s, a); break;
        case 1: hipLaunchKernelGGL((erange_kernel<T, 1>), dim3(blocks), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((erange_kernel<T, 2>), dim3(blocks), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

template hipError_t launch_step<float, float>(const StepArgs<float, float>&, int, uint64_t, int, int, int, int, size_t,
                                             hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_step<double, double>(const StepArgs<double, double>&, int, uint64_t, int, int, int, int,
                                               size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t set_step_lds_limit<float, float>(int, size_t);
template hipError_t set_step_lds_limit<double, double>(int, size_t);
template hipError_t launch_erange<float>(const ErangeArgs<float>&, int, int, hipStream_t);
template hipError_t launch_erange<double>(const ErangeArgs<double>&, int, int, hipStream_t);

}  // namespace m2m
