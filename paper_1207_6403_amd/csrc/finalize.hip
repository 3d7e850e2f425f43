// finalize.hip -- per-step reduction of the fused kernel's partial histograms.
//
// After step kernel n every (block, model) pair has written its LDS histograms
// to one partial slot.  finalize_kernel sums the slots of each column in a
// fixed order and applies, per observable j (paper section 2 and eq. 1):
//   y_j(n+1), ys_j <- ys_j + (dt/tau) (y_j - ys_j) (ys = y at the first
//   observe), Dt_j = (ys_j - Y_j)/sigma_j, the update table Dt_j/sigma_j and the
//   chunk's share of chi^2 = sum Dt_j^2;
// and per prior cell (section 2.1) the mean weight sum/count.
// Blocks never wait for each other: column blocks write per-chunk chi^2 shares
// (double-buffered by step parity), and one extra block per model assembles
// the model's statistics row of step n from the previous finalise's chi^2
// shares and step kernel n's per-slot sums; the last of them advances the
// device step counter.
#include "runtime.h"

namespace m2m {

template <typename T>
__device__ __forceinline__ T fwave_sum(T v) {
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T, typename PT>
__global__ void __launch_bounds__(256) finalize_kernel(FinArgs<T, PT> a) {
    __shared__ double part[kFinGroups][kFinCols + 1];
    __shared__ double tot[kFinCols];
    // the step failed: leave every output as it was (checked before the first
    // store, so that the loads below need not wait for the flag)
    const int failed = *a.flag;
    const int tid = threadIdx.x;
    double* chi_out = a.chunk_chi + (size_t)(a.parity) * 2 * a.nchunk;
    const double* chi_prev = a.chunk_chi + (size_t)(a.parity ^ 1) * 2 * a.nchunk;

    if ((int)blockIdx.x < a.nchunk) {
        // ------------------------------------------------ column block
        const int chunk = blockIdx.x;
        const int* d = a.chunk_desc + 8 * chunk;
        const int m = d[0], col0 = d[1], ncol = d[2], ns = d[4];
        const int64_t base = (int64_t)(uint32_t)d[5] | ((int64_t)d[6] << 32);
        const int g = tid / kFinCols, c = tid % kFinCols;
        const int col = col0 + c;
        const bool live = c < ncol && (col < a.J || (col >= a.jpad && a.accum_cells));
        // the column's target, error and smoothed value, fetched while the slots load
        const bool obs = g == 0 && live && col < a.J;
        const size_t j = (size_t)m * a.J + col;
        const double Yj = obs ? a.Y[j] : 0.0, sj = obs ? a.sigma[j] : 1.0, ysj = obs && !a.first ? a.ys[j] : 0.0;
        double acc = 0;
        if (live) {
            // slot r of the chunk at src[r * kFinCols]; group g takes r = g + kFinGroups k,
            // so that a wave reads consecutive slot rows
            const PT* src = a.part + base + c;
            for (int r0 = g; r0 < ns; r0 += kFinGroups * kSlotsPerSplit) {
                // a whole round of slots in flight before the first add
                PT v[kSlotsPerSplit];
                // unconditional loads (rows past the end re-read the last row and
                // are dropped), so that no load waits for the one before it
                #pragma unroll
                for (int k = 0; k < kSlotsPerSplit; ++k) {
                    const int r = r0 + kFinGroups * k;
                    const PT t = src[(size_t)min(r, ns - 1) * kFinCols];
                    v[k] = r < ns ? t : PT(0);
                }
                #pragma unroll
                for (int k = 0; k < kSlotsPerSplit; ++k) acc += double(v[k]);
            }
        }
        if (failed) return;
        part[g][c] = acc;
        __syncthreads();
        double chi = 0, chii = 0;
        if (g == 0) {
            double v = 0;
            #pragma unroll
            for (int k = 0; k < kFinGroups; ++k) v += part[k][c];
            tot[c] = v;
        }
        __syncthreads();
        if (g == 0 && live) {
            const double v = tot[c];
            if (col < a.J) {
                const double ys = a.first ? v : ysj + a.g * (v - ysj);
                const double dl = (ys - Yj) / sj;
                const double di = (v - Yj) / sj;
                a.y[j] = v;
                a.ys[j] = ys;
                a.delta[j] = dl;
                a.cvec[j] = T(dl / sj);
                chi = dl * dl;
                chii = di * di;
            } else if (((col - a.jpad) & 1) == 0) {
                // (sum, count) pairs never straddle a chunk: chunks start at
                // multiples of kFinCols and the cell region at an even column
                const int cell = (col - a.jpad) >> 1;
                const double cnt = tot[c + 1];
                const double mean = cnt > 0 ? v / cnt : 0.0;
                a.cellmean[(size_t)m * a.ncell + cell] = T(mean);
                a.cellmean64[(size_t)m * a.ncell + cell] = mean;
            }
        }
        if (tid < 64) {
            chi = fwave_sum(chi);
            chii = fwave_sum(chii);
            if (tid == 0) {
                chi_out[2 * chunk] = chi;
                chi_out[2 * chunk + 1] = chii;
            }
        }
        return;
    }

    // ------------------------------------------- statistics block of model m
    // (one per model; every load of the row is issued before the first wait)
    if (a.first || failed) return;
    const int m = blockIdx.x - a.nchunk;
    const long long n = a.d_step[0];
    const int c0 = a.model_chunk[m], c1 = a.model_chunk[m + 1];
    const int q0 = a.model_slot[m], q1 = a.model_slot[m + 1];
    double x2 = 0, x2i = 0, S = 0, W = 0, W2 = 0, mn = INFINITY;
    for (int k = c0 + tid; k < c1; k += 256) {
        x2 += chi_prev[2 * k];
        x2i += chi_prev[2 * k + 1];
    }
    // the slots' rows, kStatRows per thread in flight before the first wait
    constexpr int kStatRows = 4;
    const double2* rows = reinterpret_cast<const double2*>(a.seg_stats);
    for (int r0 = q0, r1 = q1; r0 < r1; r0 += 256 * kStatRows) {
        double2 v0[kStatRows], v1[kStatRows];
        #pragma unroll
        for (int u = 0; u < kStatRows; ++u) {
            const int q = r0 + u * 256 + tid;
            v0[u] = q < r1 ? rows[2 * q] : make_double2(0.0, 0.0);
            v1[u] = q < r1 ? rows[2 * q + 1] : make_double2(0.0, INFINITY);
        }
        #pragma unroll
        for (int u = 0; u < kStatRows; ++u) {
            S += v0[u].x;
            W += v0[u].y;
            W2 += v1[u].x;
            mn = fmin(mn, v1[u].y);
        }
    }
    x2 = fwave_sum(x2); x2i = fwave_sum(x2i); S = fwave_sum(S); W = fwave_sum(W); W2 = fwave_sum(W2);
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
    __shared__ double sred[6][4];
    if ((tid & 63) == 0) {
        const int w = tid >> 6;
        sred[0][w] = x2; sred[1][w] = x2i; sred[2][w] = S; sred[3][w] = W; sred[4][w] = W2; sred[5][w] = mn;
    }
    __syncthreads();
    if (tid == 0) {
        const double X2 = (sred[0][0] + sred[0][1]) + (sred[0][2] + sred[0][3]);
        const double X2i = (sred[1][0] + sred[1][1]) + (sred[1][2] + sred[1][3]);
        const double Ss = (sred[2][0] + sred[2][1]) + (sred[2][2] + sred[2][3]);
        const double Ws = (sred[3][0] + sred[3][1]) + (sred[3][2] + sred[3][3]);
        const double W2s = (sred[4][0] + sred[4][1]) + (sred[4][2] + sred[4][3]);
        const double mns = fmin(fmin(sred[5][0], sred[5][1]), fmin(sred[5][2], sred[5][3]));
        StatRow* r = a.ring + (size_t)m * kRing + (n % kRing);
        r->chi2 = X2;
        r->chi2_inst = X2i;
        r->S = Ss;
        r->F = -0.5 * X2 + a.mu * Ss;
        r->sum_w = Ws;
        r->min_w = mns;
        r->sum_w2 = W2s;
        r->n_eff = Ws * Ws / W2s;
        r->step = n;
        r->model = m;
        // the last statistics block to finish (every block has read the step
        // counter before its ticket) advances the counter and resets the tickets
        const unsigned long long ticket = __hip_atomic_fetch_add(
            reinterpret_cast<unsigned long long*>(a.d_step + 1), 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (ticket == (unsigned long long)(a.n_models - 1)) {
            a.d_step[1] = 0;
            a.d_step[0] = n + 1;
        }
    }
}

template <typename T, typename PT>
hipError_t launch_finalize(const FinArgs<T, PT>& a, hipStream_t s) {
    hipLaunchKernelGGL((finalize_kernel<T, PT>), dim3(a.nchunk + a.n_models), dim3(256), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_finalize<float, float>(const FinArgs<float, float>&, hipStream_t);
template hipError_t launch_finalize<double, double>(const FinArgs<double, double>&, hipStream_t);

}  // namespace m2m
