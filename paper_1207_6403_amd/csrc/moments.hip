// moments.hip -- velocity second moments of one model's weighted particles in
// spherical shells, from which its anisotropy profile
// beta(r) = 1 - (<v_theta^2> + <v_phi^2>) / (2 <v_r^2>) follows (paper section 3,
// Fig. 1: the anisotropy a fit recovers for a spherical target).
//
// A read-only pass over the model's rows of the current state: each block keeps
// its shell sums in LDS (FP64), writes them to its own partial row, and a second
// one-block kernel adds the rows in block order.  All arithmetic is FP64 on the
// stored coordinates, so FP32 and FP64 states are read alike.
#include <hip/hip_runtime.h>

#include "forms.h"

namespace m2m {

template <typename T>
__global__ void __launch_bounds__(kShellThreads) shell_moments_kernel(ShellArgs<T> a) {
    extern __shared__ __align__(16) double sm[];
    double* edges = sm;                          // nshell + 1
    double* acc = sm + a.nshell + 1;             // 4 x nshell
    const int ns = a.nshell, tid = threadIdx.x;
    for (int k = tid; k <= ns; k += blockDim.x) edges[k] = a.edges[k];
    for (int k = tid; k < 4 * ns; k += blockDim.x) acc[k] = 0.0;
    __syncthreads();
    const double rlo = edges[0], rhi = edges[ns];
    const int64_t S = a.stride;
    for (int64_t p = a.p0 + (int64_t)blockIdx.x * blockDim.x + tid; p < a.p1; p += (int64_t)gridDim.x * blockDim.x) {
        const double x = a.state[p], y = a.state[S + p], z = a.state[2 * S + p];
        const double vx = a.state[3 * S + p], vy = a.state[4 * S + p], vz = a.state[5 * S + p];
        const double w = a.state[6 * S + p];
        const double R2 = x * x + y * y, r = sqrt(R2 + z * z);
        if (!(r >= rlo && r < rhi)) continue;
        // shell k: edges[k] <= r < edges[k + 1]
        int lo = 0, hi = ns;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (edges[mid] <= r) lo = mid; else hi = mid;
        }
        const double vr = (x * vx + y * vy + z * vz) / r;
        const double vphi = R2 > 0.0 ? (x * vy - y * vx) / sqrt(R2) : 0.0;
        const double v2 = vx * vx + vy * vy + vz * vz;
        atomicAdd(&acc[lo], w);
        atomicAdd(&acc[ns + lo], w * vr * vr);
        atomicAdd(&acc[2 * ns + lo], w * (v2 - vr * vr - vphi * vphi));
        atomicAdd(&acc[3 * ns + lo], w * vphi * vphi);
    }
    __syncthreads();
    for (int k = tid; k < 4 * ns; k += blockDim.x) a.part[(size_t)blockIdx.x * 4 * ns + k] = acc[k];
}

__global__ void shell_sum_kernel(const double* part, int nblk, int n, double* out) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)b * n + k];
        out[k] = s;
    }
}

template <typename T>
hipError_t launch_shell_moments(const ShellArgs<T>& a, int blocks, double* out, hipStream_t s) {
    const size_t lds = sizeof(double) * (5 * (size_t)a.nshell + 1);
    hipLaunchKernelGGL(shell_moments_kernel<T>, dim3(blocks), dim3(kShellThreads), lds, s, a);
    hipLaunchKernelGGL(shell_sum_kernel, dim3(1), dim3(256), 0, s, (const double*)a.part, blocks, 4 * a.nshell, out);
    return hipGetLastError();
}

template hipError_t launch_shell_moments<float>(const ShellArgs<float>&, int, double*, hipStream_t);
template hipError_t launch_shell_moments<double>(const ShellArgs<double>&, int, double*, hipStream_t);

}  // namespace m2m
