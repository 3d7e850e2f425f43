// step.hip -- fused M2M step kernel and the per-step reduction/finalise kernel.
//
// One launch of step_kernel performs, for every particle of every model (the
// per-timestep loop of the made-to-measure method, section 2 of the paper):
//   weight update with the current deviations and priors (maximising
//   F = -chi^2/2 + mu S, eq. 1 and 2), kick-drift-kick push in the analytic
//   potential, and the scatter of w * K_j of the new state into LDS-privatised
//   observable histograms, plus the moving-prior cell sums (section 2.1).
// Each block owns a contiguous range of tiles; a tile never straddles models.
// When a block moves to another model (batched form) or finishes, it writes
// its LDS histograms to its own partial slot (no atomics, deterministic).
//
// finalize.hip then sums the partial slots column by column in a fixed order.
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

// Block-wide sum / min of four per-thread statistics into out[0..3] (thread 0).
__device__ __forceinline__ void block_stats(double s, double w, double w2, double mn, double* red, double* out) {
    s = wave_sum(s); w = wave_sum(w); w2 = wave_sum(w2); mn = wave_min(mn);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) { red[4 * wid] = s; red[4 * wid + 1] = w; red[4 * wid + 2] = w2; red[4 * wid + 3] = mn; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0, c = 0, d = INFINITY;
        for (int i = 0; i < nw; ++i) { a += red[4 * i]; b += red[4 * i + 1]; c += red[4 * i + 2]; d = fmin(d, red[4 * i + 3]); }
        out[0] = a; out[1] = b; out[2] = c; out[3] = d;
    }
    __syncthreads();
}

template <typename T, typename PT, int POT, int ILP>
__global__ void __launch_bounds__(sizeof(T) == 8 ? 256 : 512) step_kernel(StepArgs<T, PT> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (*a.flag) return;   // an earlier step failed: the whole step is a no-op

    const int J = a.lay.J, NC = a.cells.ncell, JP = a.jpad, NE = (a.nedge + 1) & ~1;
    double* hist = reinterpret_cast<double*>(smem);                 // J (padded to JP)
    double* csum = hist + JP;                                        // NC
    double* ed64 = csum + NC;                                        // edges, FP64
    double* red = ed64 + NE;                                         // 4 * 16
    const int NET = (sizeof(T) == 4 && NC) ? kLcE : 0;
    float2* et = reinterpret_cast<float2*>(red + 64);                // uniform-E Lc table (FP32)
    unsigned* ccnt = reinterpret_cast<unsigned*>(et + NET);          // NC (padded to even)
    T* cl = reinterpret_cast<T*>(ccnt + ((NC + 1) & ~1));            // J : Dt_j / sigma_j
    T* cm = cl + JP;                                                 // NC: cell means
    T* ed = cm + ((NC + 1) & ~1);                                    // edges in T
    T* lct = ed + NE;                                                // circular-orbit energies

    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < a.nedge; i += nt) { ed[i] = a.edges[i]; ed64[i] = a.ex.edges[i]; }

    const int t0 = a.block_tile0[blockIdx.x], t1 = a.block_tile0[blockIdx.x + 1];
    const bool observe_only = a.mode == 1;
    const bool want_cm = a.what_mode == 1 || a.what_mode == 2;
    int slot = a.block_slot0[blockIdx.x] - 1;
    int cur = -1;
    Pot<T> pot;
    T Emin = 0, sE = 1, wflat = 0;
    double sS = 0, sW = 0, sW2 = 0, mW = INFINITY;
    unsigned bad = 0;
    const T hdt = T(0.5) * a.dt, dt = a.dt, edt = a.eps * a.dt, mu = a.mu;

    for (int t = t0; t <= t1; ++t) {
        const int m = t < t1 ? a.tile_model[t] : -2;
        if (m != cur) {
            if (cur >= 0) {
                // flush the finished model's histograms to its partial slot
                __syncthreads();
                PT* dst = a.part + (size_t)slot * a.pcols;
                for (int j = tid; j < J; j += nt) dst[j] = PT(hist[j]);
                if (a.accum_cells)
                    for (int c = tid; c < NC; c += nt) { dst[JP + 2 * c] = PT(csum[c]); dst[JP + 2 * c + 1] = PT(ccnt[c]); }
                block_stats(sS, sW, sW2, mW, red, a.seg_stats + 4 * (size_t)slot);
                sS = sW = sW2 = 0; mW = INFINITY;
            }
            if (m < 0) break;
            cur = m;
            ++slot;
            pot = a.pots[m];
            Emin = a.erange[2 * m];
            sE = T(a.cells.n0) / (a.erange[2 * m + 1] - a.erange[2 * m]);
            wflat = a.flatw[m];
            __syncthreads();
            for (int j = tid; j < J; j += nt) { hist[j] = 0.0; cl[j] = a.cvec[(size_t)m * J + j]; }
            if (a.accum_cells) for (int c = tid; c < NC; c += nt) { csum[c] = 0.0; ccnt[c] = 0u; }
            if (want_cm) for (int c = tid; c < NC; c += nt) cm[c] = a.cellmean[(size_t)m * NC + c];
            if (NC) for (int i = tid; i < kLcTab; i += nt) lct[i] = a.lctab[(size_t)pot.lc_off + i];
            for (int i = tid; i < NET; i += nt)
                et[i] = make_float2(a.lcetab[2 * ((size_t)m * kLcE + i)], a.lcetab[2 * ((size_t)m * kLcE + i) + 1]);
            __syncthreads();
        }
        const int64_t p0 = a.tile_p0[t];
        const int cnt = a.tile_cnt[t];
        T px[ILP], py[ILP], pz[ILP], qx[ILP], qy[ILP], qz[ILP], pw[ILP];
        #pragma unroll
        for (int k = 0; k < ILP; ++k) {
            const int i = k * nt + tid;
            if (i < cnt) {
                const int64_t p = p0 + i;
                px[k] = a.in[p];
                py[k] = a.in[a.stride + p];
                pz[k] = a.in[2 * a.stride + p];
                qx[k] = a.in[3 * a.stride + p];
                qy[k] = a.in[4 * a.stride + p];
                qz[k] = a.in[5 * a.stride + p];
                pw[k] = a.in[6 * a.stride + p];
            }
        }
        #pragma unroll
        for (int k = 0; k < ILP; ++k) {
            const int i = k * nt + tid;
            if (i >= cnt) continue;
            const int64_t p = p0 + i;
            T x = px[k], y = py[k], z = pz[k], vx = qx[k], vy = qy[k], vz = qz[k], w = pw[k];
            T phi, ax, ay, az;
            potential<POT, T>(pot, x, y, z, phi, ax, ay, az);
            if (!observe_only) {
                // priors what_i at z_n
                T wh;
                if (a.what_mode == 0) {
                    wh = wflat;
                } else if (want_cm) {
                    const T E = T(0.5) * (vx * vx + vy * vy + vz * vz) + phi;
                    const int c = prior_cell<POT, T>(pot, lct, et, a.cells, Emin, sE, E, x, y, z, vx, vy, vz, a.ex, m);
                    wh = cm[c];
                    if (a.what_mode == 2) a.what[p] = wh;
                } else {
                    wh = a.what[p];
                }
                // dF/dw_i with the priors held fixed
                int jj[kMaxEntries];
                T K[kMaxEntries];
                kernel_entries<T>(a.lay, ed, ed64, x, y, z, vy, vz, jj, K);
                T chi = T(0);
                #pragma unroll
                for (int e = 0; e < kMaxEntries; ++e)
                    if (jj[e] >= 0) chi += K[e] * cl[jj[e]];
                const T lr = dlog(w / wh);
                const T G = -chi - mu * (lr + T(1));
                sS -= double(w) * double(lr);
                sW += double(w);
                sW2 += double(w) * double(w);
                mW = fmin(mW, double(w));
                const T wn = a.update == 1 ? w * dexp(edt * G) : w * (T(1) + edt * G);
                if (!(wn == wn) || wn == T(INFINITY) || wn == T(-INFINITY)) bad |= 2u;   // non-finite
                else if (!(wn > T(0))) bad |= 1u;                                        // w <= 0
                w = wn;
                // kick-drift-kick
                if (!a.frozen) {
                    vx += hdt * ax; vy += hdt * ay; vz += hdt * az;
                    x += dt * vx; y += dt * vy; z += dt * vz;
                    potential<POT, T>(pot, x, y, z, phi, ax, ay, az);
                    vx += hdt * ax; vy += hdt * ay; vz += hdt * az;
                }
                a.out[p] = x;
                a.out[a.stride + p] = y;
                a.out[2 * a.stride + p] = z;
                a.out[3 * a.stride + p] = vx;
                a.out[4 * a.stride + p] = vy;
                a.out[5 * a.stride + p] = vz;
                a.out[6 * a.stride + p] = w;
            }
            // observables and prior cells of the new state
            {
                int jj[kMaxEntries];
                T K[kMaxEntries];
                kernel_entries<T>(a.lay, ed, ed64, x, y, z, vy, vz, jj, K);
                #pragma unroll
                for (int e = 0; e < kMaxEntries; ++e)
                    if (jj[e] >= 0) atomicAdd(&hist[jj[e]], double(w * K[e]));
                if (a.accum_cells) {
                    const T E = T(0.5) * (vx * vx + vy * vy + vz * vz) + phi;
                    const int c = prior_cell<POT, T>(pot, lct, et, a.cells, Emin, sE, E, x, y, z, vx, vy, vz, a.ex, m);
                    atomicAdd(&csum[c], double(w));
                    atomicAdd(&ccnt[c], 1u);
                }
            }
        }
    }
    if (bad) {
        __hip_atomic_fetch_or(a.flag, (int)bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *a.bad_step = *a.d_step;
    }
}

// ---------------------------------------------------- energy range (at create)
template <typename T, int POT>
__global__ void __launch_bounds__(256) erange_kernel(ErangeArgs<T> a) {
    __shared__ double rmin[4], rmax[4];
    const int t0 = a.block_tile0[blockIdx.x], t1 = a.block_tile0[blockIdx.x + 1];
    int slot = a.block_slot0[blockIdx.x] - 1, cur = -1;
    double lo = INFINITY, hi = -INFINITY;
    Pot<T> pot;
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
            T phi, ax, ay, az;
            potential<POT, T>(pot, x, y, z, phi, ax, ay, az);
            const double E = double(T(0.5) * (vx * vx + vy * vy + vz * vz) + phi);
            lo = fmin(lo, E);
            hi = fmax(hi, E);
        }
    }
}

// ------------------------------------------ priors of the current state (readback)
template <typename T, int POT>
__global__ void __launch_bounds__(256) gather_kernel(GatherArgs<T> a) {
    const int t0 = a.block_tile0[blockIdx.x], t1 = a.block_tile0[blockIdx.x + 1];
    for (int t = t0; t < t1; ++t) {
        const int m = a.tile_model[t];
        const Pot<T> pot = a.pots[m];
        const T Emin = a.erange[2 * m], sE = T(a.cells.n0) / (a.erange[2 * m + 1] - a.erange[2 * m]);
        const T* lct = a.lctab + pot.lc_off;
        const int64_t p0 = a.tile_p0[t];
        const int cnt = a.tile_cnt[t];
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int64_t p = p0 + i;
            T wh;
            if (a.what_mode == 0) {
                wh = a.flatw[m];
            } else if (a.what_mode == 3) {
                wh = a.what[p];
            } else {
                T x = a.in[p], y = a.in[a.stride + p], z = a.in[2 * a.stride + p];
                T vx = a.in[3 * a.stride + p], vy = a.in[4 * a.stride + p], vz = a.in[5 * a.stride + p];
                T phi, ax, ay, az;
                potential<POT, T>(pot, x, y, z, phi, ax, ay, az);
                const T E = T(0.5) * (vx * vx + vy * vy + vz * vz) + phi;
                wh = a.cellmean[(size_t)m * a.cells.ncell +
                                prior_cell<POT, T>(pot, lct, (const float2*)a.lcetab + (size_t)m * kLcE, a.cells,
                                                   Emin, sE, E, x, y, z, vx, vy, vz, a.ex, m)];
            }
            a.out[p] = wh;
        }
    }
}

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_gather(const GatherArgs<T>& a, int pot_kind, int blocks, hipStream_t s) {
    switch (pot_kind) {
        case 0: hipLaunchKernelGGL((gather_kernel<T, 0>), dim3(blocks), dim3(256), 0, s, a); break;
        case 1: hipLaunchKernelGGL((gather_kernel<T, 1>), dim3(blocks), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((gather_kernel<T, 2>), dim3(blocks), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}
template hipError_t launch_gather<float>(const GatherArgs<float>&, int, int, hipStream_t);
template hipError_t launch_gather<double>(const GatherArgs<double>&, int, int, hipStream_t);

template <typename T, typename PT, int POT>
static hipError_t launch_step_pot(const StepArgs<T, PT>& a, int ilp, int blocks, int threads, size_t lds,
                                  hipStream_t s) {
    switch (ilp) {
        case 1: hipLaunchKernelGGL((step_kernel<T, PT, POT, 1>), dim3(blocks), dim3(threads), lds, s, a); break;
        case 2: hipLaunchKernelGGL((step_kernel<T, PT, POT, 2>), dim3(blocks), dim3(threads), lds, s, a); break;
        default: hipLaunchKernelGGL((step_kernel<T, PT, POT, 4>), dim3(blocks), dim3(threads), lds, s, a); break;
    }
    return hipGetLastError();
}

template <typename T, typename PT>
hipError_t launch_step(const StepArgs<T, PT>& a, int pot_kind, int ilp, int blocks, int threads, size_t lds,
                       hipStream_t s) {
    switch (pot_kind) {
        case 0: return launch_step_pot<T, PT, 0>(a, ilp, blocks, threads, lds, s);
        case 1: return launch_step_pot<T, PT, 1>(a, ilp, blocks, threads, lds, s);
        default: return launch_step_pot<T, PT, 2>(a, ilp, blocks, threads, lds, s);
    }
}

template <typename T, typename PT>
hipError_t set_step_lds_limit(int pot_kind, size_t lds) {
    const void* fns[] = {
        (const void*)step_kernel<T, PT, 0, 1>, (const void*)step_kernel<T, PT, 0, 2>, (const void*)step_kernel<T, PT, 0, 4>,
        (const void*)step_kernel<T, PT, 1, 1>, (const void*)step_kernel<T, PT, 1, 2>, (const void*)step_kernel<T, PT, 1, 4>,
        (const void*)step_kernel<T, PT, 2, 1>, (const void*)step_kernel<T, PT, 2, 2>, (const void*)step_kernel<T, PT, 2, 4>};
    (void)pot_kind;
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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

template hipError_t launch_step<float, float>(const StepArgs<float, float>&, int, int, int, int, size_t, hipStream_t);
template hipError_t launch_step<double, double>(const StepArgs<double, double>&, int, int, int, int, size_t, hipStream_t);
template hipError_t set_step_lds_limit<float, float>(int, size_t);
template hipError_t set_step_lds_limit<double, double>(int, size_t);
template hipError_t launch_erange<float>(const ErangeArgs<float>&, int, int, hipStream_t);
template hipError_t launch_erange<double>(const ErangeArgs<double>&, int, int, hipStream_t);

}  // namespace m2m
