// tracers.hip -- discrete line-of-sight velocities (section 1 lists PNe
// velocities among the data).  Reading: tracer t in bin b_t of one binning has
// the likelihood of the model's line-of-sight velocity density at its velocity,
//   L_t = sum_i w_i [bin(z_i) = b_t] phi(v_los,i; V_t, s_t),  M_b = sum_i w_i [bin(z_i) = b],
// both smoothed like the observables; lambda sum_t ln(Ls_t / Ms_(b_t)) joins the
// merit function, and the weight update gains
//   lambda (sum_{t in b(z_i)} phi(v_los,i; V_t, s_t) / Ls_t - n_(b(z_i)) / Ms_(b(z_i))).
//
//   tracer_observe    per block, chunks of particles counting-sorted by bin in
//                     LDS; each thread owns some tracers and sums w phi over its
//                     tracers' bins (no atomics on the sums), threads over bins
//                     sum the masses; per-block partial rows
//   tracer_sum        the rows' column sums in a fixed order (FP64), and per
//                     column its smoothing and update factor
//   tracer_loglike    one block, when the log-likelihood is read
//   tracer_grad       per chunk of particles counting-sorted by bin in LDS:
//                     each particle's term of G from the factors of its bin,
//                     with the tracers in LDS
// The bin of a particle is its stored tag, so the decisions are the step
// kernel's (exact at edges).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "forms.h"
#include "device.h"

namespace m2m {

constexpr int kTrcChunk = 4096;   // particles per chunk of tracer_observe and tracer_grad
constexpr int kTrcObsThreads = 1024;   // threads of tracer_observe and tracer_grad (one block per CU)

// exp(-d^2 / 2) of a tracer's Gaussian at d = (v - V) / s, from d' = (v - V) q / s:
// FP32 with q = sqrt(log2(e) / 2), so that it is one hardware base-2
// exponential of -d'^2; FP64 with q = 1 and the library exp.
__device__ __forceinline__ float trc_q(float) { return 0.849321800288019136f; }
__device__ __forceinline__ double trc_q(double) { return 1.0; }
__device__ __forceinline__ float trc_gauss(float dq) { return __builtin_amdgcn_exp2f(-(dq * dq)); }
__device__ __forceinline__ double trc_gauss(double dq) { return exp(-0.5 * dq * dq); }

// Exclusive prefix sum of cnt[0..n) in place (cnt[n] gets the total), by all
// threads of the block: contiguous runs per thread, then a scan of the run sums.
__device__ void block_exclusive_scan(uint32_t* cnt, int n, uint32_t* wsum) {
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6;
    const int per = (n + nt - 1) / nt;
    const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += cnt[b];
    // inclusive scan of the run sums within the wave
    uint32_t incl = s;
    #pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    uint32_t run = before + incl - s;
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = cnt[b];
        cnt[b] = run;
        run += c;
    }
    if (tid == nt - 1) cnt[n] = run;
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kTrcObsThreads) tracer_observe_kernel(TracerArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int ntr = a.ntr, nb = a.nb, tid = threadIdx.x, nt = blockDim.x;
    double* acc = reinterpret_cast<double*>(smem);            // ntr, each owned by one thread
    double* mass = acc + ntr;                                  // nb
    T* svl = reinterpret_cast<T*>(mass + nb);                  // kTrcChunk, sorted by bin
    T* sw = svl + kTrcChunk;                                   // kTrcChunk
    uint32_t* cnt = reinterpret_cast<uint32_t*>(sw + kTrcChunk);   // nb + 1: counts, then starts
    uint32_t* wsum = cnt + nb + 1;                             // 16
    if (*a.flag) return;
    for (int k = tid; k < ntr + nb; k += nt) acc[k] = 0.0;     // (mass follows acc)
    const uint16_t* tag = reinterpret_cast<const uint16_t*>(a.state + 7 * a.stride) + (size_t)a.tagrow * a.stride;
    const T* S = a.state;
    const int64_t st = a.stride;
    constexpr int kPer = kTrcChunk / kTrcObsThreads;
    for (int64_t c0 = (int64_t)blockIdx.x * kTrcChunk; c0 < a.n; c0 += (int64_t)gridDim.x * kTrcChunk) {
        for (int b = tid; b <= nb; b += nt) cnt[b] = 0u;
        __syncthreads();
        int bq[kPer];
        uint32_t slot[kPer];
        T vq[kPer], wq[kPer];
        // (the velocities and weight are loaded with the tag, not after it: a
        // particle in no bin leaves them unused)
        #pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int64_t p = min(c0 + tid + q * kTrcObsThreads, a.n - 1);
            bq[q] = tag[p];
            vq[q] = line_of_sight(S[4 * st + p], S[5 * st + p], a.sini, a.cosi);
            wq[q] = S[6 * st + p];
        }
        #pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const bool in = c0 + tid + q * kTrcObsThreads < a.n && bq[q] != kNoBin;
            if (in) slot[q] = atomicAdd(&cnt[bq[q]], 1u);
            else bq[q] = -1;
        }
        __syncthreads();
        block_exclusive_scan(cnt, nb, wsum);
        #pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (bq[q] >= 0) {
                const uint32_t pos = cnt[bq[q]] + slot[q];
                svl[pos] = vq[q];
                sw[pos] = wq[q];
            }
        __syncthreads();
        for (int b = tid; b < nb; b += nt) {
            double m = 0.0;
            for (uint32_t i = cnt[b]; i < cnt[b + 1]; ++i) m += double(sw[i]);
            mass[b] += m;
        }
        for (int t = tid; t < ntr; t += nt) {
            const int b = a.tbin[t];
            const T V = a.V[t], isq = a.is[t] * trc_q(T(0));
            // four particles per round, their LDS reads issued together and their
            // terms added in pairs before the FP64 sum
            double s0 = 0.0;
            uint32_t i = cnt[b];
            const uint32_t e = cnt[b + 1];
            for (; i + 4 <= e; i += 4) {
                T v[4], w[4];
                #pragma unroll
                for (int u = 0; u < 4; ++u) { v[u] = svl[i + u]; w[u] = sw[i + u]; }
                const T g0 = w[0] * trc_gauss((v[0] - V) * isq), g1 = w[1] * trc_gauss((v[1] - V) * isq);
                const T g2 = w[2] * trc_gauss((v[2] - V) * isq), g3 = w[3] * trc_gauss((v[3] - V) * isq);
                s0 += double((g0 + g1) + (g2 + g3));
            }
            for (; i < e; ++i) s0 += double(sw[i] * trc_gauss((svl[i] - V) * isq));
            acc[t] += double(a.nf[t]) * s0;   // (the tracer's normalisation, once per chunk)
        }
        __syncthreads();
    }
    double* dst = a.part + (size_t)blockIdx.x * (ntr + nb);
    for (int k = tid; k < ntr + nb; k += nt) dst[k] = acc[k];
}

// Column sums of the block rows: a block per 64 columns, its four waves each
// adding a quarter of the rows (16 loads in flight), the quarters added in wave
// order (a fixed order).
template <typename T>
__global__ void __launch_bounds__(256) tracer_sum_kernel(TracerArgs<T> a) {
    __shared__ double sh[4][64];
    if (*a.flag) return;
    const int W = a.ntr + a.nb, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane, cc = min(col, W - 1);
    double s = 0.0;
    for (int q0 = wv; q0 < a.nblk; q0 += 4 * 16) {
        double v[16];
        #pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = a.part[(size_t)min(q0 + 4 * u, a.nblk - 1) * W + cc];
        #pragma unroll
        for (int u = 0; u < 16; ++u) s += q0 + 4 * u < a.nblk ? v[u] : 0.0;
    }
    sh[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && col < W) {
        // the column's smoothing and update factor (each column is one tracer's
        // sum or one bin's mass: no other column is needed)
        const double v = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
        if (col < a.ntr) {
            const double ls = a.first_obs ? v : a.Ls[col] + a.g * (v - a.Ls[col]);
            a.Ls[col] = ls;
            a.cL_out[col] = T(a.lambda / ls);
        } else {
            const int b = col - a.ntr, nbt = a.first[b + 1] - a.first[b];
            const double ms = a.first_obs ? v : a.Ms[b] + a.g * (v - a.Ms[b]);
            a.Ms[b] = ms;
            a.cM_out[b] = nbt ? T(-a.lambda * nbt / ms) : T(0);
        }
    }
}

// The log-likelihood sum_t ln(Ls_t / Ms_(b_t)) of the smoothed sums as they
// stand (one block; launched when it is read).
template <typename T>
__global__ void __launch_bounds__(256) tracer_loglike_kernel(TracerArgs<T> a) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double ll = 0.0;
    for (int t = tid; t < a.ntr; t += 256) ll += log(a.Ls[t] / a.Ms[a.tbin[t]]);
    red[tid] = ll;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) *a.loglike = red[0];
}

// Per chunk of particles, counting-sorted by bin in LDS as in tracer_observe, so
// that the 64 lanes of a wave take consecutive particles of (mostly) one bin:
// their loops over the bin's tracers then have one length and read the same
// tracer at once.  Each particle's term goes back to its own place; particles in
// no bin get 0.
template <typename T>
__global__ void __launch_bounds__(kTrcObsThreads) tracer_grad_kernel(TracerArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int ntr = a.ntr, nb = a.nb, tid = threadIdx.x, nt = blockDim.x;
    T* tV = reinterpret_cast<T*>(smem);                          // ntr
    T* tis = tV + ntr;                                            // ntr
    T* tc = tis + ntr;                                            // ntr: cL nf
    T* svl = tc + ntr;                                            // kTrcChunk, sorted by bin
    uint16_t* sidx = reinterpret_cast<uint16_t*>(svl + kTrcChunk);   // kTrcChunk: index in the chunk
    uint16_t* sbin = sidx + kTrcChunk;                            // kTrcChunk: bin
    uint32_t* cnt = reinterpret_cast<uint32_t*>(sbin + kTrcChunk);   // nb + 1: counts, then starts
    uint32_t* wsum = cnt + nb + 1;                                // 16
    if (*a.flag) return;
    for (int t = tid; t < ntr; t += nt) {
        tV[t] = a.V[t];
        tis[t] = a.is[t] * trc_q(T(0));
        tc[t] = a.cL[t] * a.nf[t];
    }
    const uint16_t* tag = reinterpret_cast<const uint16_t*>(a.state + 7 * a.stride) + (size_t)a.tagrow * a.stride;
    const T* S = a.state;
    const int64_t st = a.stride;
    constexpr int kPer = kTrcChunk / kTrcObsThreads;
    for (int64_t c0 = (int64_t)blockIdx.x * kTrcChunk; c0 < a.n; c0 += (int64_t)gridDim.x * kTrcChunk) {
        for (int b = tid; b <= nb; b += nt) cnt[b] = 0u;
        __syncthreads();
        int bq[kPer];
        uint32_t slot[kPer];
        T vq[kPer];
        // (the velocities are loaded with the tag, not after it)
        #pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int64_t p = min(c0 + tid + q * kTrcObsThreads, a.n - 1);
            bq[q] = tag[p];
            vq[q] = line_of_sight(S[4 * st + p], S[5 * st + p], a.sini, a.cosi);
        }
        #pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int64_t p = c0 + tid + q * kTrcObsThreads;
            if (p < a.n && bq[q] != kNoBin) {
                slot[q] = atomicAdd(&cnt[bq[q]], 1u);
            } else {
                if (p < a.n) a.extra[p] = T(0);
                bq[q] = -1;
            }
        }
        __syncthreads();
        block_exclusive_scan(cnt, nb, wsum);
        #pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (bq[q] >= 0) {
                const uint32_t pos = cnt[bq[q]] + slot[q];
                svl[pos] = vq[q];
                sidx[pos] = (uint16_t)(tid + q * kTrcObsThreads);
                sbin[pos] = (uint16_t)bq[q];
            }
        __syncthreads();
        const uint32_t total = cnt[nb];
        for (uint32_t pos = tid; pos < total; pos += nt) {
            const int b = sbin[pos];
            const T vl = svl[pos];
            T x = a.cM[b], x1 = T(0);
            // four tracers per round, their LDS reads issued together, into two sums
            int t = a.first[b];
            const int te = a.first[b + 1];
            for (; t + 4 <= te; t += 4) {
                T V[4], q[4], c[4];
                #pragma unroll
                for (int u = 0; u < 4; ++u) { V[u] = tV[t + u]; q[u] = tis[t + u]; c[u] = tc[t + u]; }
                x += c[0] * trc_gauss((vl - V[0]) * q[0]);
                x1 += c[1] * trc_gauss((vl - V[1]) * q[1]);
                x += c[2] * trc_gauss((vl - V[2]) * q[2]);
                x1 += c[3] * trc_gauss((vl - V[3]) * q[3]);
            }
            for (; t < te; ++t) x += tc[t] * trc_gauss((vl - tV[t]) * tis[t]);
            a.extra[c0 + sidx[pos]] = x + x1;
        }
        __syncthreads();   // (the next chunk reuses the LDS)
    }
}

template <typename T>
static size_t observe_lds(const TracerArgs<T>& a) {
    return sizeof(double) * (size_t)(a.ntr + a.nb) + 2 * sizeof(T) * kTrcChunk + sizeof(uint32_t) * (a.nb + 1 + 16);
}

template <typename T>
hipError_t launch_tracer_observe(const TracerArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL(tracer_observe_kernel<T>, dim3(a.nblk), dim3(kTrcObsThreads), observe_lds(a), s, a);
    hipLaunchKernelGGL(tracer_sum_kernel<T>, dim3((a.ntr + a.nb + 63) / 64), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tracer_loglike(const TracerArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL(tracer_loglike_kernel<T>, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
static size_t grad_lds(const TracerArgs<T>& a) {
    return 3 * sizeof(T) * (size_t)a.ntr + (sizeof(T) + 4) * kTrcChunk + sizeof(uint32_t) * (a.nb + 1 + 16);
}

template <typename T>
hipError_t launch_tracer_grad(const TracerArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL(tracer_grad_kernel<T>, dim3(a.nblk), dim3(kTrcObsThreads), grad_lds(a), s, a);
    return hipGetLastError();
}

template <typename T>
size_t tracer_lds(const TracerArgs<T>& a) {
    return std::max(observe_lds(a), grad_lds(a));
}

template <typename T>
hipError_t set_tracer_lds_limit(size_t lds) {
    hipError_t e = hipFuncSetAttribute((const void*)tracer_observe_kernel<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)tracer_grad_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template hipError_t launch_tracer_observe<float>(const TracerArgs<float>&, hipStream_t);
template hipError_t launch_tracer_observe<double>(const TracerArgs<double>&, hipStream_t);
template hipError_t launch_tracer_loglike<float>(const TracerArgs<float>&, hipStream_t);
template hipError_t launch_tracer_loglike<double>(const TracerArgs<double>&, hipStream_t);
template hipError_t launch_tracer_grad<float>(const TracerArgs<float>&, hipStream_t);
template hipError_t launch_tracer_grad<double>(const TracerArgs<double>&, hipStream_t);
template size_t tracer_lds<float>(const TracerArgs<float>&);
template size_t tracer_lds<double>(const TracerArgs<double>&);
template hipError_t set_tracer_lds_limit<float>(size_t);
template hipError_t set_tracer_lds_limit<double>(size_t);

}  // namespace m2m
