// particle.h -- per-particle pieces shared by the step kernels (step.hip) and
// the self-consistent multipole kernels (multipole.hip): block reductions, the
// per-block working set, state-buffer addressing, and the weight update.
#pragma once
#include <type_traits>

#include "runtime.h"

namespace m2m {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// Wave sum / min of four per-thread statistics into the wave's row of out
// (out[4 w .. 4 w + 3] for wave w of the block): no block barrier.
// Weight statistics of a block, (S, sum w, sum w^2, min w): each wave reduces
// its lanes and leaves its four values in lds[4 * wave ..] before a block
// barrier the caller already has; after it, one thread adds the waves in order
// and writes the block's row (deterministic, no extra barrier).
__device__ __forceinline__ void wave_stats(double s, double w, double w2, double mn, double* lds) {
    s = wave_sum(s); w = wave_sum(w); w2 = wave_sum(w2); mn = wave_min(mn);
    if ((threadIdx.x & 63) == 0) {
        double* o = lds + 4 * (threadIdx.x >> 6);
        o[0] = s; o[1] = w; o[2] = w2; o[3] = mn;
    }
}
__device__ __forceinline__ void block_stats_write(const double* lds, int nwave, double* out) {
    double s = 0.0, w = 0.0, w2 = 0.0, mn = INFINITY;
    for (int k = 0; k < nwave; ++k) {
        s += lds[4 * k];
        w += lds[4 * k + 1];
        w2 += lds[4 * k + 2];
        mn = fmin(mn, lds[4 * k + 3]);
    }
    out[0] = s; out[1] = w; out[2] = w2; out[3] = mn;
}

// Per-block working set of one model (LDS tables and model constants).
template <typename T>
struct Blk {
    double* hist;       // observable histogram (FP64)
    double* csum;       // prior cell weight sums
    unsigned* ccnt;     // prior cell counts
    const T* cl;        // update table Dt_j / sigma_j
    const T* cm;        // prior cell means
    const T* ed;        // edges in T
    const double* ed64; // edges in FP64
    const float2* et;   // uniform-E Lc table (FP32 kernels)
    const T* lct;       // circular-orbit energies (FP64 kernels)
    const T* gh;        // Gauss-Hermite (V, 1/sigma) pairs of the layout's GH bins
    Pot<T> pot;
    T Emin, sE, wflat;
    CellGuard cg;       // energy-axis guard of the prior cells (FP32 kernels)
    int m;
};

// Statistics of the weights entering the step, accumulated per thread.
struct Acc {
    double S = 0, W = 0, W2 = 0, mn = INFINITY;
    unsigned bad = 0;
};

// Element i of a table that no kernel writes while it runs, read through the
// constant address space: uniform indices then become scalar loads, which do
// not wait behind the vector stores of the particle loop.
template <typename X>
__device__ __forceinline__ X ro(const X* p, int64_t i) {
    if constexpr (std::is_arithmetic<X>::value) {
        return ((const __attribute__((address_space(4))) X*)p)[i];
    } else {
        // a struct, word by word
        static_assert(sizeof(X) % 4 == 0, "whole words");
        X v;
        const __attribute__((address_space(4))) uint32_t* s = (const __attribute__((address_space(4))) uint32_t*)(p + i);
        uint32_t* d = reinterpret_cast<uint32_t*>(&v);
        #pragma unroll
        for (unsigned k = 0; k < sizeof(X) / 4; ++k) d[k] = s[k];
        return v;
    }
}

// Pull every 64-byte line of the kernel's argument block into the scalar cache
// in one round trip (one word per line, all loads issued before the first
// wait): the compiler places each argument load next to its first use, and
// those loads then hit the cache instead of waiting on memory one after the
// other.
template <int BYTES>
__device__ __forceinline__ void warm_kernargs() {
    using cU32 = const __attribute__((address_space(4))) uint32_t;
    cU32* k = (cU32*)__builtin_amdgcn_kernarg_segment_ptr();
    constexpr int kLines = (BYTES + 63) / 64;
    uint32_t v[kLines];
    #pragma unroll
    for (int i = 0; i < kLines; ++i) v[i] = k[16 * i];
    #pragma unroll
    for (int i = 0; i < kLines; ++i) asm volatile("" ::"s"(v[i]));
}

// Value at byte offset off from base.  Every row of a state buffer (values,
// then tags) is addressed from the buffer's base with a 32-bit byte offset
// (state buffers are smaller than 4 GiB), so one scalar base serves all rows.
template <typename X>
__device__ __forceinline__ X ld_at(const void* base, uint32_t off) {
    return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) + off);
}
template <typename X>
__device__ __forceinline__ void st_at(void* base, uint32_t off, X v) {
    *reinterpret_cast<X*>(reinterpret_cast<char*>(base) + off) = v;
}

// Scatter w * K_j of one particle's bin k of binning b (moments of v_los = vl);
// when take is false the terms go to the lane's trash slot instead.
// (Gauss-Hermite moments read the bin's (V, 1/sigma) pair from gh; a particle
// outside the binning reads pair 0 for a value that goes to the trash slot.)
template <uint64_t SIG, typename T>
__device__ __forceinline__ void scatter_bin(const LayoutView<SIG, T>& V, double* hist, int b, int k, bool take,
                                            int trash, T wn, T vl, const T* gh) {
    const BinDesc<T>& d = V.L.b[b];
    const int base = d.off + k;
    const int nmom = V.nmom(b), mom = V.mom(b);
    const T* gv = gh + 2 * (d.gh0 + (k < 0 ? 0 : k));
    #pragma unroll
    for (int mm = 0; mm < 3; ++mm) {
        if (mm >= nmom) break;
        const int code = (mom >> (kMomBits * mm)) & 7;
        const T kv = V.has_gh() ? kernel_value<T>(code, vl, gv) : moment_value<T>(code, vl);
        atomicAdd(&hist[take ? base + mm * d.nb : trash], double(wn * kv));
    }
}

// w(n+1) of one particle (section 2: dw/dt = eps w dF/dw with F of eq. 1 and S
// of eq. 2, the priors held fixed; exp law w exp(eps dt G) or Euler w (1 + eps
// dt G)), from the kernel entries of its stored bins and the update table;
// accumulates the statistics of w(n) and stores the prior a refresh step used.
// ZSLOT >= 0: B.cl[ZSLOT] is zero, and bins without a particle read it instead
// of branching (the fused kernel's LDS table); ZSLOT < 0: they are skipped.
template <int NB, uint64_t SIG, int ZSLOT = -1, typename T, typename PT>
__device__ __forceinline__ T weight_update(const StepArgs<T, PT>& a, const Blk<T>& B, Acc& acc, int64_t p, T vy, T vz,
                                           T w, T what_p, const uint16_t (&tg)[kMaxBin + 1], uint32_t fl, int zslot = 0) {
    const Layout<T>& L = a.lay;
    const LayoutView<SIG, T> V{L};
    const int nbin = V.nbin();
    const T vl = line_of_sight(vy, vz, L.sini, L.cosi);
    T chi = T(-0.0);   // (adding -0 is exact for every value, so the first sum folds away)
    #pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nbin) break;
        const int k = tg[b];
        if constexpr (ZSLOT < 0) {
            if (k == kNoBin) continue;
        }
        const int base = L.b[b].off + k;
        const int nmom = V.nmom(b), mom = V.mom(b);
        const T* gv = B.gh + 2 * (L.b[b].gh0 + (k == kNoBin ? 0 : k));
        #pragma unroll
        for (int mm = 0; mm < 3; ++mm) {
            if (mm >= nmom) break;
            const int j = (ZSLOT >= 0 && k == kNoBin) ? zslot : base + mm * L.b[b].nb;
            const int code = (mom >> (kMomBits * mm)) & 7;
            const T kv = V.has_gh() ? kernel_value<T>(code, vl, gv) : moment_value<T>(code, vl);
            chi += kv * B.cl[j];
        }
    }
    const uint32_t wm = (fl >> kWhatShift) & 3u;
    const T wh = wm == 0 ? B.wflat : (wm == 3 ? what_p : B.cm[tg[kMaxBin]]);
    // (FP32: the hardware log, exp and reciprocal, a few ulp each; the FP64
    // kernels use the exact forms)
    const T lr = qlog_ratio(qdiv(w, wh));
    const T G = -chi - a.mu * (lr + T(1)) + ((fl & kTracers) ? a.extra[p] : T(-0.0));
    const T edt = a.eps * a.dt;
    const T wn = (fl & kExpLaw) ? w * qexp(edt * G) : w * (T(1) + edt * G);
    acc.S -= double(w) * double(lr);
    acc.W += double(w);
    acc.W2 += double(w) * double(w);
    acc.mn = fmin(acc.mn, double(w));
    if (!(wn == wn) || wn == T(INFINITY) || wn == T(-INFINITY)) acc.bad |= 2u;   // non-finite
    else if (!(wn > T(0))) acc.bad |= 1u;                                        // w <= 0
    if (wm == 2) a.what[p] = wh;   // a refresh step stores the prior it used
    return wn;
}

}  // namespace m2m
