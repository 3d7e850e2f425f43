// mlp.hip -- the learned moving prior (section 2.1: priors that follow the
// structure of the weight distribution over integrals of motion, here a smooth
// function of them fitted to the weights).
//
// Every `period` steps, before the step's update, one refresh runs
//   mlp_subset    a Philox4x32-10 sample of the particles: features
//                 u = (2 (E - Emin)/(Emax - Emin) - 1, 2 L/Lc(E) - 1, Lz/L) (FP64
//                 integrals, FP32 features) and the target ln w
//   mlp_train     per minibatch: forward and backward of each sample (eight
//                 threads per sample), the block's gradient sums (32 samples
//                 per block)
//   mlp_adam      the minibatch gradient (block sums in block order) and one Adam
//                 step (Kingma & Ba 2015, Algorithm 1)
//   mlp_infer     g(u) of every particle, per-block maxima
//   mlp_norm      e = exp(g - max g), per-block sums of e and w
//   mlp_judge     what = e sum w / sum e, per-block sums of w |ln what - ln what_hist|
//   mlp_select    the histogram prior instead when the w-weighted mean exceeds
//                 the fallback threshold
// with single-block reductions of the per-block partials in between, in block
// order (deterministic).
#include <mutex>

#include "forms.h"

namespace m2m {

// ------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror & Shaw (2011): ten rounds of two 32x32 -> 64-bit
// multiplications on a 4-word counter under a 2-word key bumped by the Weyl
// constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    #pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0), hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Features of the particle at row offset p of the state (FP64 integrals of the
// FP32 coordinates), and its weight.
template <int POT>
__device__ __forceinline__ void mlp_features(const MlpArgs& a, int64_t p, float& u0, float& u1, float& u2, float& w) {
    const float* s = a.state;
    const int64_t S = a.stride;
    const double x = s[p], y = s[S + p], z = s[2 * S + p], vx = s[3 * S + p], vy = s[4 * S + p], vz = s[5 * S + p];
    w = s[6 * S + p];
    const Exact* ex = a.ex;
    double E, L, Lz, Lc;
    integrals_seeded<POT>(ex->pots[0], ex->lctab, ex->rce, double(a.lcE0), double(a.lcEinv), x, y, z, vx, vy, vz, E, L,
                          Lz, Lc);
    u0 = float(2.0 * (E - a.Emin) / (a.Emax - a.Emin) - 1.0);
    u1 = float(Lc > 0.0 ? 2.0 * L / Lc - 1.0 : -1.0);
    u2 = float(L > 0.0 ? Lz / L : 0.0);
}

// The FP64 features out of line (the rare FP64 route of the FP32 features below,
// kept out of the register allocation of the kernels that call it).
template <int POT>
__device__ __noinline__ float4 mlp_features_ool(const MlpArgs& a, int64_t p) {
    float4 f;
    mlp_features<POT>(a, p, f.x, f.y, f.z, f.w);
    return f;
}

// The same features in FP32 for the BF16 inference (whose network rounds its
// activations to 8 bits, so FP32 integrals lose nothing): the FP32 potential,
// L and Lz, and Lc(E) from the uniform-E table; an energy outside the table
// takes the FP64 route.
template <int POT>
__device__ __forceinline__ void mlp_features32(const MlpArgs& a, int64_t p, float& u0, float& u1, float& u2,
                                               float& w) {
    const float* s = a.state;
    const int64_t S = a.stride;
    const float x = s[p], y = s[S + p], z = s[2 * S + p], vx = s[3 * S + p], vy = s[4 * S + p], vz = s[5 * S + p];
    w = s[6 * S + p];
    const Pot<float> pt = *a.pot32;
    float phi, ax, ay, az;
    potential<POT, float>(pt, x, y, z, phi, ax, ay, az);
    const float E = 0.5f * (vx * vx + vy * vy + vz * vz) + phi;
    const float lx = y * vz - z * vy, ly = z * vx - x * vz, lz = x * vy - y * vx;
    const float L = sqrtf(lx * lx + ly * ly + lz * lz);
    float Lc, dl;
    if (!lc_from_table(a.lcetab, pt.lcE0, pt.lcEinv, E, 0.0f, Lc, dl)) {
        const float4 f = mlp_features_ool<POT>(a, p);
        u0 = f.x; u1 = f.y; u2 = f.z; w = f.w;
        return;
    }
    u0 = float(2.0 * (double(E) - a.Emin) / (a.Emax - a.Emin) - 1.0);
    u1 = Lc > 0.0f ? 2.0f * L / Lc - 1.0f : -1.0f;
    u2 = L > 0.0f ? lz / L : 0.0f;
}

template <int POT>
__global__ void __launch_bounds__(256) mlp_subset_kernel(MlpArgs a) {
    if (*a.flag) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.subset) return;
    uint32_t c[4] = {uint32_t(k >> 2), a.q, 0u, 0u};
    philox4x32_10(c, a.seed, 0u);
    const uint32_t word = c[k & 3];
    const int64_t p = int64_t(((uint64_t)word * (uint64_t)a.n) >> 32);
    float u0, u1, u2, w;
    mlp_features<POT>(a, p, u0, u1, u2, w);
    a.sub[k] = make_float4(u0, u1, u2, logf(w));
}

// Operand vectors of the matrix-core products (v_mfma_f32_16x16x32_bf16: lane l
// holds row l % 16 and k = 8 (l / 16) .. + 7 of A, column l % 16 and the same k of
// B, and column l % 16, rows 4 (l / 16) .. + 3 of the FP32 result).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// tanh(x) = 1 - 2 / (exp(2x) + 1), with the hardware exp and reciprocal: an
// absolute error of a few 1e-7 over the whole line (+-1 in the limits), which
// is what the units' sums see.
__device__ __forceinline__ float unit_tanh(float x) {
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * x) + 1.0f);
}
// The BF16 inference's form: its weights and biases come pre-multiplied by
// 2 log2(e), so that y = 2 log2(e) x and 1 / (exp(2x) + 1) is one hardware base-2
// exponential, an add and a reciprocal (tanh(x) = 1 - 2 r).
constexpr float kTwoLog2e = 2.88539008177792681f;
__device__ __forceinline__ float unit_r(float y) { return __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y) + 1.0f); }

// Forward pass of one sample with the parameters th in LDS: the first hidden
// layer h1 (registers), the second layer's units one by one (to h2, an LDS row,
// when given) and the output g.
__device__ __forceinline__ float mlp_forward(const float* th, float u0, float u1, float u2, float (&h1)[kMlpH],
                                             float* h2) {
    #pragma unroll
    for (int o = 0; o < kMlpH; ++o)
        h1[o] = unit_tanh(th[kMlpB1 + o] + th[kMlpW1 + 3 * o] * u0 + th[kMlpW1 + 3 * o + 1] * u1 + th[kMlpW1 + 3 * o + 2] * u2);
    float g = th[kMlpB3];
    #pragma unroll 2
    for (int o = 0; o < kMlpH; ++o) {
        const float4* row = reinterpret_cast<const float4*>(th + kMlpW2 + kMlpH * o);
        float acc = th[kMlpB2 + o];
        #pragma unroll
        for (int i = 0; i < kMlpH / 4; ++i) {
            const float4 r = row[i];
            acc += r.x * h1[4 * i] + r.y * h1[4 * i + 1] + r.z * h1[4 * i + 2] + r.w * h1[4 * i + 3];
        }
        const float t = unit_tanh(acc);
        if (h2) h2[o] = t;
        g += th[kMlpW3 + o] * t;
    }
    return g;
}

// Minibatch b, block of kMlpSamples samples (b*batch + blockIdx.x*kMlpSamples on),
// kMlpTPS threads per sample: thread t takes sample s = t / kMlpTPS and the units
// q*UPT .. q*UPT+UPT-1 (q = t % kMlpTPS, UPT = 64 / kMlpTPS) of each layer; activations and deltas are shared
// in LDS.  Loss (g - t)^2 averaged over the minibatch.  The block's gradient sums
// over its samples (in sample order) go to its partial row.  W2 is held in LDS
// with rows padded to kW2Row floats, so that the eight rows a wave reads at once
// fall in different banks.
constexpr int kW2Row = kMlpH + 4;
constexpr int kThW2 = kMlpB1 + kMlpH;                    // W2 in the LDS copy
constexpr int kThB2 = kThW2 + kMlpH * kW2Row;
constexpr int kThW3 = kThB2 + kMlpH, kThB3 = kThW3 + kMlpH, kThN = kThB3 + 4;
constexpr int kActRow = kMlpH + 1;

// Copy the parameters into a block's LDS with all of a thread's loads issued
// before the first wait (a load-then-store loop waits once per element).
template <int NT, typename Put>
__device__ __forceinline__ void load_theta(const float* __restrict__ theta, Put&& put) {
    constexpr int kPer = (kMlpNP + NT - 1) / NT;
    float v[kPer];
    #pragma unroll
    for (int u = 0; u < kPer; ++u) v[u] = theta[min(int(threadIdx.x) + u * NT, kMlpNP - 1)];
    #pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = int(threadIdx.x) + u * NT;
        if (i < kMlpNP) put(i, v[u]);
    }
}

__global__ void __launch_bounds__(kMlpTrainThreads) mlp_train_kernel(MlpArgs a, int b) {
    __shared__ __align__(16) float th[kThN];
    __shared__ float H1[kMlpSamples][kActRow], H2[kMlpSamples][kActRow];
    __shared__ float D2[kMlpSamples][kActRow], D1[kMlpSamples][kActRow];
    __shared__ float U[kMlpSamples][4];
    if (*a.flag) return;
    const int tid = threadIdx.x, s = tid / kMlpTPS, q = tid % kMlpTPS;
    constexpr int UPT = kMlpH / kMlpTPS;   // units per thread
    // the sample first: its load is then in flight with the parameters'
    const float4 smp = a.sub[(size_t)b * a.batch + (size_t)blockIdx.x * kMlpSamples + s];
    load_theta<kMlpTrainThreads>(a.theta, [&](int i, float v) {
        int d;
        if (i < kMlpW2) d = i;
        else if (i < kMlpB2) d = kThW2 + ((i - kMlpW2) / kMlpH) * kW2Row + (i - kMlpW2) % kMlpH;
        else d = kThB2 + (i - kMlpB2);
        th[d] = v;
    });
    __syncthreads();
    // layer 1
    #pragma unroll
    for (int k = 0; k < UPT; ++k) {
        const int o = q * UPT + k;
        H1[s][o] = unit_tanh(th[kMlpB1 + o] + th[kMlpW1 + 3 * o] * smp.x + th[kMlpW1 + 3 * o + 1] * smp.y +
                             th[kMlpW1 + 3 * o + 2] * smp.z);
    }
    __syncthreads();
    // layer 2 and the output
    float acc[UPT];
    #pragma unroll
    for (int k = 0; k < UPT; ++k) acc[k] = th[kThB2 + q * UPT + k];
    for (int i = 0; i < kMlpH; i += 4) {
        const float h0 = H1[s][i], h1 = H1[s][i + 1], h2 = H1[s][i + 2], h3 = H1[s][i + 3];
        #pragma unroll
        for (int k = 0; k < UPT; ++k) {
            const float4 r = *reinterpret_cast<const float4*>(&th[kThW2 + (q * UPT + k) * kW2Row + i]);
            acc[k] += r.x * h0 + r.y * h1 + r.z * h2 + r.w * h3;
        }
    }
    float gp = 0.0f;
    #pragma unroll
    for (int k = 0; k < UPT; ++k) {
        acc[k] = unit_tanh(acc[k]);
        gp += th[kThW3 + q * UPT + k] * acc[k];
    }
    #pragma unroll
    for (int o = kMlpTPS / 2; o > 0; o >>= 1) gp += __shfl_xor(gp, o, 64);   // the sample's kMlpTPS threads, in a fixed tree
    const float g = th[kThB3] + gp;
    const float dg = 2.0f * (g - smp.w) / float(a.batch);
    if (a.loss && q == 0) a.loss[(size_t)blockIdx.x * kMlpSamples + s] = (g - smp.w) * (g - smp.w) / float(a.batch);
    #pragma unroll
    for (int k = 0; k < UPT; ++k) {
        const int o = q * UPT + k;
        H2[s][o] = acc[k];
        D2[s][o] = dg * th[kThW3 + o] * (1.0f - acc[k] * acc[k]);
    }
    if (q == 0) { U[s][0] = smp.x; U[s][1] = smp.y; U[s][2] = smp.z; U[s][3] = dg; }
    __syncthreads();
    // back to layer 1: d1 = (W2^T d2) (1 - h1^2)
    float d1[UPT];
    #pragma unroll
    for (int k = 0; k < UPT; ++k) d1[k] = 0.0f;
    for (int o = 0; o < kMlpH; ++o) {
        const float d2 = D2[s][o];
        #pragma unroll
        for (int k = 0; k < UPT; ++k) d1[k] += th[kThW2 + o * kW2Row + q * UPT + k] * d2;
    }
    #pragma unroll
    for (int k = 0; k < UPT; ++k) {
        const int i = q * UPT + k;
        const float h = H1[s][i];
        D1[s][i] = d1[k] * (1.0f - h * h);
    }
    __syncthreads();
    // sums over the block's samples: kTPR threads per W2 row, thread t takes row
    // o = t / kTPR, columns kCols (t % kTPR) .. +kCols-1; threads t < 64 also row
    // t of b2, W3, b1, W1, thread 0 b3
    float* dst = a.gpart + (size_t)blockIdx.x * kMlpNP;
    {
        constexpr int kTPR = kMlpTrainThreads / kMlpH, kCols = kMlpH / kTPR;
        static_assert(kTPR * kMlpH == kMlpTrainThreads && kCols * kTPR == kMlpH, "W2 rows split evenly");
        const int o = tid / kTPR, i0 = kCols * (tid % kTPR);
        float gw[kCols];
        #pragma unroll
        for (int j = 0; j < kCols; ++j) gw[j] = 0.0f;
        for (int ss = 0; ss < kMlpSamples; ++ss) {
            const float d2 = D2[ss][o];
            #pragma unroll
            for (int j = 0; j < kCols; ++j) gw[j] += d2 * H1[ss][i0 + j];
        }
        #pragma unroll
        for (int j = 0; j < kCols; ++j) dst[kMlpW2 + kMlpH * o + i0 + j] = gw[j];
    }
    if (tid < kMlpH) {
        const int o = tid;
        float gb2 = 0.0f, gw3 = 0.0f, gb1 = 0.0f, gw10 = 0.0f, gw11 = 0.0f, gw12 = 0.0f;
        for (int ss = 0; ss < kMlpSamples; ++ss) {
            const float d2 = D2[ss][o], d1o = D1[ss][o];
            gb2 += d2;
            gw3 += U[ss][3] * H2[ss][o];
            gb1 += d1o;
            gw10 += d1o * U[ss][0];
            gw11 += d1o * U[ss][1];
            gw12 += d1o * U[ss][2];
        }
        dst[kMlpB2 + o] = gb2;
        dst[kMlpW3 + o] = gw3;
        dst[kMlpB1 + o] = gb1;
        dst[kMlpW1 + 3 * o] = gw10;
        dst[kMlpW1 + 3 * o + 1] = gw11;
        dst[kMlpW1 + 3 * o + 2] = gw12;
        if (o == 0) {
            float gb3 = 0.0f;
            for (int ss = 0; ss < kMlpSamples; ++ss) gb3 += U[ss][3];
            dst[kMlpB3] = gb3;
        }
    }
}

// The same training step with the three 32 x 64 x 64 contractions of a block on
// the matrix cores (BF16 operands, FP32 accumulation): 256 threads (four waves)
// per block of 32 samples.  Wave w takes
//   the forward hidden layer  Z2[s][o] = sum_i H1[s][i] W2[o][i]   for units 16w..16w+15,
//   the backward to layer 1   D1[s][i] = sum_o D2[s][o] W2[o][i]   for inputs 16w..16w+15,
//   the W2 gradient           dW2[o][i] = sum_s D2[s][o] H1[s][i]  for units 16w..16w+15,
// each as 16x16x32 products (the W2 slices it needs held in registers as BF16);
// the elementwise layers, the output and the other parameters' sums are FP32 on
// the VALU.  Operands in LDS: activations and deltas per sample (BF16 rows) and
// transposed (BF16 rows per unit), FP32 copies for the elementwise work.
constexpr int kTrainMfmaThreads = 256;
constexpr int kRowB = kMlpH + 8;              // BF16 row of 64 units (padded)
constexpr int kRowT = kMlpSamples + 8;        // BF16 row of 32 samples (padded)

__global__ void __launch_bounds__(kTrainMfmaThreads) mlp_train_mfma_kernel(MlpArgs a, int b) {
    constexpr int S = kMlpSamples, H = kMlpH;
    __shared__ float w1s[H][4];                         // W1 row and b1 per unit
    __shared__ float b2s[H], w3s[H];
    __shared__ float U[S][4];                           // u0 u1 u2 and dg per sample
    __shared__ float H1f[S][H + 1], H2f[S][H + 1], D2f[S][H + 1], D1f[S][H + 1];
    __shared__ __align__(16) __bf16 H1b[S][kRowB], D2b[S][kRowB];
    __shared__ __align__(16) __bf16 H1T[H][kRowT], D2T[H][kRowT];
    if (*a.flag) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int l16 = lane & 15, q4 = lane >> 4;
    const size_t s0 = (size_t)b * a.batch + (size_t)blockIdx.x * S;
    for (int o = tid; o < H; o += kTrainMfmaThreads) {
        w1s[o][0] = a.theta[kMlpW1 + 3 * o];
        w1s[o][1] = a.theta[kMlpW1 + 3 * o + 1];
        w1s[o][2] = a.theta[kMlpW1 + 3 * o + 2];
        w1s[o][3] = a.theta[kMlpB1 + o];
        b2s[o] = a.theta[kMlpB2 + o];
        w3s[o] = a.theta[kMlpW3 + o];
    }
    if (tid < S) {
        const float4 smp = a.sub[s0 + tid];
        U[tid][0] = smp.x; U[tid][1] = smp.y; U[tid][2] = smp.z; U[tid][3] = smp.w;
    }
    // W2 slices: forward (rows 16w + l16, inputs 32 k + 8 q4 + v) and backward
    // (units 32 k + 8 q4 + v, input column 16w + l16)
    bf16x8 wf[2], wb[2];
    #pragma unroll
    for (int k = 0; k < 2; ++k)
        #pragma unroll
        for (int v = 0; v < 8; ++v) {
            wf[k][v] = (__bf16)a.theta[kMlpW2 + (16 * wv + l16) * H + 32 * k + 8 * q4 + v];
            wb[k][v] = (__bf16)a.theta[kMlpW2 + (32 * k + 8 * q4 + v) * H + 16 * wv + l16];
        }
    const float b3 = a.theta[kMlpB3];
    __syncthreads();
    // layer 1: thread takes sample tid / 8 and units 8 (tid % 8) .. + 7
    {
        const int s = tid >> 3, o0 = 8 * (tid & 7);
        bf16x8 hv;
        #pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int o = o0 + v;
            const float h = unit_tanh(w1s[o][3] + w1s[o][0] * U[s][0] + w1s[o][1] * U[s][1] + w1s[o][2] * U[s][2]);
            H1f[s][o] = h;
            hv[v] = (__bf16)h;
            H1T[o][s] = (__bf16)h;
        }
        *reinterpret_cast<bf16x8*>(&H1b[s][o0]) = hv;
    }
    __syncthreads();
    // forward hidden layer: units 16 wv + l16 of samples 16 t + 4 q4 + v
    #pragma unroll
    for (int t = 0; t < 2; ++t) {
        floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        #pragma unroll
        for (int k = 0; k < 2; ++k)
            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(&H1b[16 * t + l16][32 * k + 8 * q4]),
                                                        wf[k], z, 0, 0, 0);
        const int o = 16 * wv + l16;
        #pragma unroll
        for (int v = 0; v < 4; ++v) H2f[16 * t + 4 * q4 + v][o] = unit_tanh(z[v] + b2s[o]);
    }
    __syncthreads();
    // output and its derivative per sample
    if (tid < S) {
        float g = b3;
        for (int o = 0; o < H; ++o) g += w3s[o] * H2f[tid][o];
        const float dg = 2.0f * (g - U[tid][3]) / float(a.batch);
        if (a.loss) a.loss[(size_t)blockIdx.x * S + tid] = (g - U[tid][3]) * (g - U[tid][3]) / float(a.batch);
        U[tid][3] = dg;
    }
    __syncthreads();
    {
        const int s = tid >> 3, o0 = 8 * (tid & 7);
        bf16x8 dv;
        #pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int o = o0 + v;
            const float h = H2f[s][o];
            const float d = U[s][3] * w3s[o] * (1.0f - h * h);
            D2f[s][o] = d;
            dv[v] = (__bf16)d;
            D2T[o][s] = (__bf16)d;
        }
        *reinterpret_cast<bf16x8*>(&D2b[s][o0]) = dv;
    }
    __syncthreads();
    // back to layer 1: inputs 16 wv + l16 of samples 16 t + 4 q4 + v
    #pragma unroll
    for (int t = 0; t < 2; ++t) {
        floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        #pragma unroll
        for (int k = 0; k < 2; ++k)
            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(&D2b[16 * t + l16][32 * k + 8 * q4]),
                                                        wb[k], z, 0, 0, 0);
        const int i = 16 * wv + l16;
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int s = 16 * t + 4 * q4 + v;
            const float h = H1f[s][i];
            D1f[s][i] = z[v] * (1.0f - h * h);
        }
    }
    // W2 gradient: units 16 wv + 4 q4 + v, inputs 16 c + l16 (one product over the 32 samples)
    float* dst = a.gpart + (size_t)blockIdx.x * kMlpNP;
    {
        const bf16x8 af = *reinterpret_cast<const bf16x8*>(&D2T[16 * wv + l16][8 * q4]);
        #pragma unroll
        for (int c = 0; c < 4; ++c) {
            floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, *reinterpret_cast<const bf16x8*>(&H1T[16 * c + l16][8 * q4]), z,
                                                        0, 0, 0);
            #pragma unroll
            for (int v = 0; v < 4; ++v) dst[kMlpW2 + (16 * wv + 4 * q4 + v) * H + 16 * c + l16] = z[v];
        }
    }
    __syncthreads();
    if (tid < H) {
        const int o = tid;
        float gb2 = 0.0f, gw3 = 0.0f, gb1 = 0.0f, gw10 = 0.0f, gw11 = 0.0f, gw12 = 0.0f;
        for (int ss = 0; ss < S; ++ss) {
            const float d2 = D2f[ss][o], d1o = D1f[ss][o];
            gb2 += d2;
            gw3 += U[ss][3] * H2f[ss][o];
            gb1 += d1o;
            gw10 += d1o * U[ss][0];
            gw11 += d1o * U[ss][1];
            gw12 += d1o * U[ss][2];
        }
        dst[kMlpB2 + o] = gb2;
        dst[kMlpW3 + o] = gw3;
        dst[kMlpB1 + o] = gb1;
        dst[kMlpW1 + 3 * o] = gw10;
        dst[kMlpW1 + 3 * o + 1] = gw11;
        dst[kMlpW1 + 3 * o + 2] = gw12;
        if (o == 0) {
            float gb3 = 0.0f;
            for (int ss = 0; ss < S; ++ss) gb3 += U[ss][3];
            dst[kMlpB3] = gb3;
        }
    }
}

// Sum of the training blocks' partial rows for parameter j = 64 blockIdx.x +
// lane, in a fixed order (FP64): wave w of the 16 adds rows w, w + 16, ...
// (16 rows in flight per round), then the wave sums are added in wave order.
constexpr int kSumWaves = 16;
__device__ __forceinline__ bool grad_row_sum(const MlpArgs& a, int nblk, double* part, float& g) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    const int jj = min(j, kMlpNP - 1);
    double gs = 0.0;
    for (int k0 = w; k0 < nblk; k0 += kSumWaves * 16) {
        float v[16];
        #pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = a.gpart[(size_t)min(k0 + kSumWaves * u, nblk - 1) * kMlpNP + jj];
        #pragma unroll
        for (int u = 0; u < 16; ++u) gs += k0 + kSumWaves * u < nblk ? double(v[u]) : 0.0;
    }
    part[w * 64 + lane] = gs;
    __syncthreads();
    if (w != 0 || j >= kMlpNP) return false;
    double t = part[lane];
    for (int k = 1; k < kSumWaves; ++k) t += part[k * 64 + lane];
    g = float(t);
    return true;
}

// One Adam step on the minibatch gradient; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void __launch_bounds__(64 * kSumWaves) mlp_adam_kernel(MlpArgs a, int nblk, float c1, float c2) {
    __shared__ double part[kSumWaves * 64];
    if (*a.flag) return;
    float g;
    if (!grad_row_sum(a, nblk, part, g)) return;
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const float m = a.beta1 * a.adam_m[j] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.adam_v[j] + (1.0f - a.beta2) * g * g;
    a.adam_m[j] = m;
    a.adam_v[j] = v;
    a.theta[j] -= a.lr * (m / c1) / (sqrtf(v / c2) + a.adam_eps);
}

// The minibatch gradient alone (the blocks' rows added as in mlp_adam_kernel).
__global__ void __launch_bounds__(64 * kSumWaves) mlp_grad_sum_kernel(MlpArgs a, int nblk, float* grad) {
    __shared__ double part[kSumWaves * 64];
    float g;
    if (grad_row_sum(a, nblk, part, g)) grad[blockIdx.x * 64 + (threadIdx.x & 63)] = g;
}

// Block partials of the inference passes: thread values reduced in a fixed tree.
__device__ __forceinline__ double block_reduce(double v, bool is_max, double* sh) {
    const int tid = threadIdx.x;
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o, 64);
        v = is_max ? fmax(v, u) : v + u;
    }
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int k = 1; k < int(blockDim.x >> 6); ++k) r = is_max ? fmax(r, sh[k]) : r + sh[k];
    __syncthreads();
    return r;
}

template <int POT>
__global__ void __launch_bounds__(kMlpInferThreads, 2) mlp_infer_kernel(MlpArgs a) {
    __shared__ __align__(16) float th[kMlpNP + 3];
    __shared__ double sh[kMlpInferThreads / 64];
    if (*a.flag) return;
    const int tid = threadIdx.x;
    load_theta<kMlpInferThreads>(a.theta, [&](int i, float v) { th[i] = v; });
    __syncthreads();
    double gmax = -INFINITY;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + tid; p < a.n; p += (int64_t)gridDim.x * blockDim.x) {
        float u0, u1, u2, w;
        mlp_features<POT>(a, p, u0, u1, u2, w);
        float h1[kMlpH];
        // (the parameters are read from LDS for every particle rather than held
        // in registers across the loop, which would leave one wave per SIMD)
        const float g = mlp_forward(th + opaque(0u), u0, u1, u2, h1, nullptr);
        a.what[p] = g;
        gmax = fmax(gmax, double(g));
    }
    gmax = block_reduce(gmax, true, sh);
    if (tid == 0) a.red[2 * blockIdx.x] = gmax;
}

// The same inference with the 64 x 64 hidden layer on the matrix cores (BF16
// operands, FP32 accumulation): each wave takes 64 particles, one per lane for
// the features and the first layer, whose outputs go to an LDS row per particle
// as BF16; the hidden layer is then 4 x 4 tiles of 16 particles x 16 units, each
// two 16x16x32 BF16 products (units' W2 rows held in registers as BF16), and each
// lane finishes the tanh and the output sum for its units of 16 particles; the
// 16 lanes that share particles add their partial outputs.
constexpr int kHRow = kMlpH + 8;   // LDS row of one particle's first-layer outputs (BF16, padded)

// Sum over the 16 lanes of a row (lanes 16 r .. 16 r + 15), the same in every
// lane of the row: with data-parallel-primitive moves, the pairs and the quads
// (quad permutations 1 0 3 2 and 2 3 0 1), then the halves of the row (the
// half-row mirror takes lane i of eight from lane 7 - i) and the row (the row
// mirror: lane 15 - i).
__device__ __forceinline__ float row_sum16(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false));
    return x;
}

// P32: the features in FP32 (four waves per SIMD: the FP64 route is out of
// line), else in FP64 (two).
template <int POT, bool P32>
__global__ void __launch_bounds__(kMlpInferThreads, P32 ? 4 : 2) mlp_infer_mfma_kernel(MlpArgs a) {
    constexpr int kWaves = kMlpInferThreads / 64;
    __shared__ __align__(16) float l1[kMlpH][4];               // W1 row and b1 per unit
    __shared__ float b2s[kMlpH], w3s[kMlpH];
    __shared__ __align__(16) __bf16 hrow[kWaves][64][kHRow];
    __shared__ float gbuf[kWaves][64];
    __shared__ double sh[kMlpInferThreads / 64];
    if (*a.flag) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // the hidden layers' weights and biases times 2 log2(e) (unit_r), and -2 w3:
    // a unit's output term w3 tanh(x) = w3 - 2 w3 r
    for (int o = tid; o < kMlpH; o += kMlpInferThreads) {
        l1[o][0] = kTwoLog2e * a.theta[kMlpW1 + 3 * o];
        l1[o][1] = kTwoLog2e * a.theta[kMlpW1 + 3 * o + 1];
        l1[o][2] = kTwoLog2e * a.theta[kMlpW1 + 3 * o + 2];
        l1[o][3] = kTwoLog2e * a.theta[kMlpB1 + o];
        b2s[o] = kTwoLog2e * a.theta[kMlpB2 + o];
        w3s[o] = -2.0f * a.theta[kMlpW3 + o];
    }
    // B operands: unit n = 16 c + lane % 16, inputs k = 32 s + 8 (lane / 16) + v
    bf16x8 bw[4][2];
    #pragma unroll
    for (int c = 0; c < 4; ++c)
        #pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
            #pragma unroll
            for (int v = 0; v < 8; ++v)
                bw[c][s2][v] =
                    (__bf16)(kTwoLog2e * a.theta[kMlpW2 + (16 * c + (lane & 15)) * kMlpH + 32 * s2 + 8 * (lane >> 4) + v]);
    const float b3 = a.theta[kMlpB3];
    // the sum of w3 over this lane's four units (their w3 terms, added once)
    float w3l = 0.0f;
    #pragma unroll
    for (int c = 0; c < 4; ++c) w3l += a.theta[kMlpW3 + 16 * c + (lane & 15)];
    __syncthreads();
    double gmax = -INFINITY;
    for (int64_t base = (int64_t)blockIdx.x * kMlpInferThreads; base < a.n; base += (int64_t)gridDim.x * kMlpInferThreads) {
        const int64_t p = base + tid;
        float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f, w;
        if (p < a.n) {
            if constexpr (P32) mlp_features32<POT>(a, p, u0, u1, u2, w);
            else mlp_features<POT>(a, p, u0, u1, u2, w);
        }
        // first layer, to this particle's LDS row in BF16
        #pragma unroll
        for (int o8 = 0; o8 < kMlpH; o8 += 8) {
            bf16x8 hv;
            #pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int o = o8 + v;
                hv[v] = (__bf16)fmaf(-2.0f, unit_r(l1[o][3] + l1[o][0] * u0 + l1[o][1] * u1 + l1[o][2] * u2), 1.0f);
            }
            *reinterpret_cast<bf16x8*>(&hrow[wv][lane][o8]) = hv;
        }
        __syncthreads();
        #pragma unroll
        for (int t = 0; t < 4; ++t) {
            // (the products accumulate onto the units' biases: every element a lane
            // holds belongs to its unit 16 c + lane % 16)
            floatx4 acc[4];
            #pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float b = b2s[16 * c + (lane & 15)];
                acc[c] = floatx4{b, b, b, b};
            }
            #pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const bf16x8 af = *reinterpret_cast<const bf16x8*>(&hrow[wv][16 * t + (lane & 15)][32 * s2 + 8 * (lane >> 4)]);
                #pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bw[c][s2], acc[c], 0, 0, 0);
            }
            // lane holds units 16 c + lane % 16 of particles 16 t + 4 (lane / 16) + v;
            // the 16 lanes that hold the same particles (one row) add their sums
            #pragma unroll
            for (int v = 0; v < 4; ++v) {
                float x = w3l;
                #pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int n = 16 * c + (lane & 15);
                    x = fmaf(w3s[n], unit_r(acc[c][v]), x);
                }
                x = row_sum16(x);
                if ((lane & 15) == 0) gbuf[wv][16 * t + 4 * (lane >> 4) + v] = x + b3;
            }
        }
        __syncthreads();
        if (p < a.n) {
            const float g = gbuf[wv][lane];
            a.what[p] = g;
            gmax = fmax(gmax, double(g));
        }
        __syncthreads();
    }
    gmax = block_reduce(gmax, true, sh);
    if (tid == 0) a.red[2 * blockIdx.x] = gmax;
}

__global__ void __launch_bounds__(kMlpInferThreads) mlp_norm_kernel(MlpArgs a) {
    __shared__ double sh[kMlpInferThreads / 64];
    if (*a.flag) return;
    const float gmax = float(a.stats[0]);
    const float* wrow = a.state + 6 * a.stride;
    double se = 0.0, sw = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * blockDim.x) {
        const float e = expf(a.what[p] - gmax);
        a.what[p] = e;
        se += double(e);
        sw += double(wrow[p]);
    }
    se = block_reduce(se, false, sh);
    sw = block_reduce(sw, false, sh);
    if (threadIdx.x == 0) {
        a.red[2 * blockIdx.x] = sw;
        a.red[2 * blockIdx.x + 1] = se;
    }
}

__global__ void __launch_bounds__(kMlpInferThreads) mlp_judge_kernel(MlpArgs a) {
    __shared__ double sh[kMlpInferThreads / 64];
    if (*a.flag) return;
    const float scale = float(a.stats[1] / a.stats[2]);
    const float* wrow = a.state + 6 * a.stride;
    const uint16_t* cell = reinterpret_cast<const uint16_t*>(a.state + 7 * a.stride) + (size_t)a.cellrow * a.stride;
    double sj = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * blockDim.x) {
        const float what = a.what[p] * scale;
        a.what[p] = what;
        const float hist = a.cellmean[cell[p]];
        sj += double(wrow[p]) * fabs(log(double(what)) - log(double(hist)));
    }
    sj = block_reduce(sj, false, sh);
    if (threadIdx.x == 0) a.red[2 * blockIdx.x] = sj;
}

__global__ void __launch_bounds__(kMlpInferThreads) mlp_select_kernel(MlpArgs a) {
    if (*a.flag || a.stats[5] == 0.0) return;
    const uint16_t* cell = reinterpret_cast<const uint16_t*>(a.state + 7 * a.stride) + (size_t)a.cellrow * a.stride;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * blockDim.x)
        a.what[p] = a.cellmean[cell[p]];
}

// Reductions of the per-block partials (one block; thread t takes partials t,
// t + 256, ... in order, then a fixed tree):
//   0: stats[0] = max g;  1: stats[1] = sum w, stats[2] = sum e;
//   2: stats[3] = sum w |ln what - ln what_hist|, stats[4] = its w-weighted mean,
//      stats[5] = 1 when that exceeds the fallback threshold, stats[6] += 1.
__global__ void __launch_bounds__(256) mlp_reduce_kernel(MlpArgs a, int mode) {
    __shared__ double sh[2][256];
    if (*a.flag) return;
    const int tid = threadIdx.x;
    const bool is_max = mode == 0;
    double u = is_max ? -INFINITY : 0.0, v = 0.0;
    for (int k = tid; k < a.nblk; k += 256) {
        if (is_max) u = fmax(u, a.red[2 * k]);
        else { u += a.red[2 * k]; v += a.red[2 * k + 1]; }
    }
    sh[0][tid] = u;
    sh[1][tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            sh[0][tid] = is_max ? fmax(sh[0][tid], sh[0][tid + o]) : sh[0][tid] + sh[0][tid + o];
            sh[1][tid] += sh[1][tid + o];
        }
        __syncthreads();
    }
    if (tid != 0) return;
    if (mode == 0) {
        a.stats[0] = sh[0][0];
    } else if (mode == 1) {
        a.stats[1] = sh[0][0];
        a.stats[2] = sh[1][0];
    } else {
        a.stats[3] = sh[0][0];
        a.stats[4] = sh[0][0] / a.stats[1];
        a.stats[5] = a.stats[4] > a.fallback ? 1.0 : 0.0;
        a.stats[6] += 1.0;
    }
}

template <int POT>
static hipError_t refresh_pot(const MlpArgs& a, int t0, hipStream_t s) {
    hipError_t e;
    hipLaunchKernelGGL((mlp_subset_kernel<POT>), dim3((a.subset + 255) / 256), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nb = a.subset / a.batch, nblk = a.batch / kMlpSamples;
    for (int b = 0; b < nb; ++b) {
        const int t = t0 + b + 1;
        const float c1 = float(1.0 - std::pow(double(a.beta1), t)), c2 = float(1.0 - std::pow(double(a.beta2), t));
        if (a.mfma) hipLaunchKernelGGL(mlp_train_mfma_kernel, dim3(nblk), dim3(kTrainMfmaThreads), 0, s, a, b);
        else hipLaunchKernelGGL(mlp_train_kernel, dim3(nblk), dim3(kMlpTrainThreads), 0, s, a, b);
        hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpNP + 63) / 64), dim3(64 * kSumWaves), 0, s, a, nblk, c1, c2);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (a.mfma && a.pot32) hipLaunchKernelGGL((mlp_infer_mfma_kernel<POT, true>), dim3(a.nblk), dim3(kMlpInferThreads), 0, s, a);
    else if (a.mfma) hipLaunchKernelGGL((mlp_infer_mfma_kernel<POT, false>), dim3(a.nblk), dim3(kMlpInferThreads), 0, s, a);
    else hipLaunchKernelGGL((mlp_infer_kernel<POT>), dim3(a.nblk), dim3(kMlpInferThreads), 0, s, a);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(1), dim3(256), 0, s, a, 0);
    hipLaunchKernelGGL(mlp_norm_kernel, dim3(a.nblk), dim3(kMlpInferThreads), 0, s, a);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(1), dim3(256), 0, s, a, 1);
    hipLaunchKernelGGL(mlp_judge_kernel, dim3(a.nblk), dim3(kMlpInferThreads), 0, s, a);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(1), dim3(256), 0, s, a, 2);
    hipLaunchKernelGGL(mlp_select_kernel, dim3(a.nblk), dim3(kMlpInferThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpArgs& a, float* grad, hipStream_t s) {
    const int nblk = a.batch / kMlpSamples;
    if (a.mfma) hipLaunchKernelGGL(mlp_train_mfma_kernel, dim3(nblk), dim3(kTrainMfmaThreads), 0, s, a, 0);
    else hipLaunchKernelGGL(mlp_train_kernel, dim3(nblk), dim3(kMlpTrainThreads), 0, s, a, 0);
    hipLaunchKernelGGL(mlp_grad_sum_kernel, dim3((kMlpNP + 63) / 64), dim3(64 * kSumWaves), 0, s, a, nblk, grad);
    return hipGetLastError();
}

// ------------------------------------------- loss and gradient without allocation
// The working memory of launch_mlp_grad_noalloc: the training blocks' partial
// gradient rows, then the per-sample loss terms, for at most kMlpNoAllocMax
// samples.  Each device that runs the library holds one copy until the process
// ends.  Host code never uses this name as an address: the device address comes
// from hipGetSymbolAddress (mlp_noalloc_scratch).
static __device__ __align__(256) float scratch[kMlpNoAllocFloats];

namespace {
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t mlp_noalloc_scratch(int device, float** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        // (the caller has made `device` current)
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// Sum of the n per-sample loss terms in FP64: thread t adds terms t, t + 256, ...
// in order, then a fixed tree.
__global__ void __launch_bounds__(256) mlp_loss_sum_kernel(const float* terms, int n, double* out) {
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    double v = 0.0;
    for (int k = tid; k < n; k += 256) v += double(terms[k]);
    sh[tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) sh[tid] += sh[tid + o];
        __syncthreads();
    }
    if (tid == 0) *out = sh[0];
}

hipError_t launch_mlp_grad_noalloc(MlpArgs a, float* scratch_ptr, float* grad, double* loss, hipStream_t s) {
    a.gpart = scratch_ptr;
    a.loss = scratch_ptr + (size_t)(kMlpNoAllocMax / kMlpSamples) * kMlpNP;
    const hipError_t e = launch_mlp_grad(a, grad, s);
    if (e != hipSuccess || !loss) return e;
    hipLaunchKernelGGL(mlp_loss_sum_kernel, dim3(1), dim3(256), 0, s, a.loss, a.batch, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_refresh(const MlpArgs& a, int pot_kind, int t0, hipStream_t s) {
    switch (pot_kind) {
        case 0: return refresh_pot<0>(a, t0, s);
        case 1: return refresh_pot<1>(a, t0, s);
        default: return refresh_pot<2>(a, t0, s);
    }
}

}  // namespace m2m
