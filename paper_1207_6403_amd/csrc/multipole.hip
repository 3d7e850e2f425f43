// multipole.hip -- the self-consistent potential of the particles (sections 1
// and 2 of the paper: the potential may be computed from the particle model
// itself), as a multipole expansion to l <= lmax of the masses m_i = w_i Mtot:
//   Phi(x) = -G sum_lm c_lm [Re Y_lm (Ac r^-(l+1) + Bc r^l) + Im Y_lm (As r^-(l+1) + Bs r^l)]
// with Y_lm = P_l^m(cos t) e^(i m ph) (Condon-Shortley phase), c_lm =
// (2 - d_m0)(l-m)!/(l+m)!, A_lm(r) = sum_{r_k < r} m_k r_k^l Y_lm(k) and
// B_lm(r) = sum_{r_k >= r} m_k r_k^-(l+1) Y_lm(k) (cos and sin parts).  A and B are
// kept at nn log-spaced node radii in [rmin, rmax] (per-interval sums, then a
// prefix scan for A and a suffix scan for B) and interpolated linearly in ln r;
// radii outside [rmin, rmax] are evaluated at the clamped radius.
//
// One step of a multipole model runs
//   mp_kick_drift   weight update, first half kick (the field at x_n, stored by the
//                   previous step's second kick), drift
//   per-interval sums of the drifted particles with the new weights: FP32
//                   mp_interval, mp_offsets, mp_scatter (counting sort by
//                   interval), mp_accum, mp_chunksum; FP64 mp_coeff_atomic
//   mp_scan         node coefficients of step n+1
//   mp_kick         second half kick; stores the field at x_n+1 for the next step
// then the fused step kernel observing the new state, and the finalise kernel.
#include <hip/hip_ext.h>

#include "particle.h"
#include "forms.h"

namespace m2m {

constexpr int kMpTri = (kMpL + 1) * (kMpL + 2) / 2;   // (l, m >= 0) pairs

__host__ __device__ constexpr int tri(int l, int m) { return l * (l + 1) / 2 + m; }
// index of the cos (s = 0) or sin (s = 1) coefficient of (l, m) in the tables
__host__ __device__ constexpr int lm_at(int l, int m, int s) { return m == 0 ? l * l : l * l + 2 * m - 1 + s; }
__host__ __device__ constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
__host__ __device__ constexpr double mp_c(int l, int m) { return (m == 0 ? 1.0 : 2.0) * fact(l - m) / fact(l + m); }

// Y_lm of the unit vector u for l <= lmax: P_m^m = (-1)^m (2m-1)!! st^m, so
// Y_mm = -(2m-1)(ux + i uy) Y_(m-1)(m-1); Y_(m+1)m = (2m+1) uz Y_mm; then the
// recurrence in l, (l-m) Y_lm = (2l-1) uz Y_(l-1)m - (l+m-1) Y_(l-2)m.
template <typename T>
__device__ __forceinline__ void mp_harmonics(T ux, T uy, T uz, T (&Yr)[kMpTri], T (&Yi)[kMpTri]) {
    Yr[0] = T(1);
    Yi[0] = T(0);
    #pragma unroll
    for (int m = 0; m <= kMpL; ++m) {
        if (m > 0) {
            const T pr = Yr[tri(m - 1, m - 1)], pi = Yi[tri(m - 1, m - 1)], f = -T(2 * m - 1);
            Yr[tri(m, m)] = f * (ux * pr - uy * pi);
            Yi[tri(m, m)] = f * (ux * pi + uy * pr);
        }
        if (m + 1 <= kMpL) {
            Yr[tri(m + 1, m)] = T(2 * m + 1) * uz * Yr[tri(m, m)];
            Yi[tri(m + 1, m)] = T(2 * m + 1) * uz * Yi[tri(m, m)];
        }
        #pragma unroll
        for (int l = m + 2; l <= kMpL; ++l) {
            const T inv = T(1.0 / (l - m));
            Yr[tri(l, m)] = (T(2 * l - 1) * uz * Yr[tri(l - 1, m)] - T(l + m - 1) * Yr[tri(l - 2, m)]) * inv;
            Yi[tri(l, m)] = (T(2 * l - 1) * uz * Yi[tri(l - 1, m)] - T(l + m - 1) * Yi[tri(l - 2, m)]) * inv;
        }
    }
}

// Recurrence and expansion constants by (l, m) for a loop over l that is not
// fully unrolled (its index is uniform, so these are scalar loads rather than
// conversions): (2l-1)/(l-m), (l+m-1)/(l-m), c_lm = (2 - d_m0)(l-m)!/(l+m)!, l+m
// and -(l+m)(l+m-1) (the derivative factors), and by l: 2l-1 and 2l+1.
struct MpConst {
    float a[kMpL + 1][kMpL + 1], b[kMpL + 1][kMpL + 1], c[kMpL + 1][kMpL + 1];
    float s[kMpL + 1][kMpL + 1], d[kMpL + 1][kMpL + 1], o[kMpL + 1], p[kMpL + 1];
    double ad[kMpL + 1][kMpL + 1], bd[kMpL + 1][kMpL + 1], cd[kMpL + 1][kMpL + 1];
    double sd[kMpL + 1][kMpL + 1], dd[kMpL + 1][kMpL + 1], od[kMpL + 1], pd[kMpL + 1];
};
constexpr MpConst make_mp_const() {
    MpConst k{};
    for (int l = 0; l <= kMpL; ++l)
        for (int m = 0; m <= l; ++m) {
            const double a = l - m >= 2 ? double(2 * l - 1) / (l - m) : 0.0;
            const double b = l - m >= 2 ? double(l + m - 1) / (l - m) : 0.0;
            k.a[l][m] = float(a); k.b[l][m] = float(b); k.c[l][m] = float(mp_c(l, m));
            k.ad[l][m] = a; k.bd[l][m] = b; k.cd[l][m] = mp_c(l, m);
            k.s[l][m] = float(l + m); k.sd[l][m] = l + m;
            k.d[l][m] = -float((l + m) * (l + m - 1)); k.dd[l][m] = -double((l + m) * (l + m - 1));
        }
    for (int l = 0; l <= kMpL; ++l) {
        k.o[l] = float(2 * l - 1); k.od[l] = 2 * l - 1;
        k.p[l] = float(2 * l + 1); k.pd[l] = 2 * l + 1;
    }
    return k;
}
__constant__ MpConst kMpC = make_mp_const();

template <typename T>
__device__ __forceinline__ T mpk_a(int l, int m) { if constexpr (sizeof(T) == 4) return kMpC.a[l][m]; else return kMpC.ad[l][m]; }
template <typename T>
__device__ __forceinline__ T mpk_b(int l, int m) { if constexpr (sizeof(T) == 4) return kMpC.b[l][m]; else return kMpC.bd[l][m]; }
template <typename T>
__device__ __forceinline__ T mpk_c(int l, int m) { if constexpr (sizeof(T) == 4) return kMpC.c[l][m]; else return kMpC.cd[l][m]; }
template <typename T>
__device__ __forceinline__ T mpk_s(int l, int m) { if constexpr (sizeof(T) == 4) return kMpC.s[l][m]; else return kMpC.sd[l][m]; }
template <typename T>
__device__ __forceinline__ T mpk_d(int l, int m) { if constexpr (sizeof(T) == 4) return kMpC.d[l][m]; else return kMpC.dd[l][m]; }
template <typename T>
__device__ __forceinline__ T mpk_o(int l) { if constexpr (sizeof(T) == 4) return kMpC.o[l]; else return kMpC.od[l]; }
template <typename T>
__device__ __forceinline__ T mpk_p(int l) { if constexpr (sizeof(T) == 4) return kMpC.p[l]; else return kMpC.pd[l]; }

// Copy of the FP32 node table (n float4 entries) into LDS by the block's nt
// threads: each thread issues its kMpCopyRounds loads before the first LDS
// write, so that the copy costs one memory round trip, not one per entry (the
// largest table that fits LDS needs ten rounds of 1024 threads).
constexpr int kMpCopyRounds = 10;
__device__ __forceinline__ void mp_table_to_lds(float4* __restrict__ dst, const float4* __restrict__ src, int n,
                                                int tid, int nt) {
    for (int i0 = tid; i0 < n; i0 += kMpCopyRounds * nt) {
        float4 v[kMpCopyRounds];
        // indexes past the end re-read the last entry and write it back to its
        // place (unconditional writes: no write waits in a branch of its own)
        #pragma unroll
        for (int k = 0; k < kMpCopyRounds; ++k) v[k] = src[min(i0 + k * nt, n - 1)];
        #pragma unroll
        for (int k = 0; k < kMpCopyRounds; ++k) dst[min(i0 + k * nt, n - 1)] = v[k];
    }
}

// Potential and acceleration at (x, y, z) from a node table tab (FP64: nn nodes
// of kMpW values, A then B; FP32: nn nodes of kMpRowF values, 16-byte (A cos,
// B cos, A sin, B sin) entries by (l, m); the terms above the model's lmax are
// zero), the
// coefficients held fixed at the interpolated values.  With R_lm = r^l Y_lm the
// gradient follows from d/dz R_lm = (l+m) R_(l-1)m, (d/dx + i d/dy) R_lm =
// R_(l-1)(m+1) and (d/dx - i d/dy) R_lm = -(l+m)(l+m-1) R_(l-1)(m-1) (m >= 1; the
// conjugate of the former for m = 0), and is free of the polar-axis
// singularity of spherical coordinates.  The loop runs over l with the rows
// Y_l*, Y_(l-1)*, Y_(l-2)* in registers.
template <typename T, typename TabT>
__device__ __forceinline__ void mp_field(const MpArgs<T>& mp, const TabT* __restrict__ tab, T x, T y, T z, T& phi,
                                         T& ax, T& ay, T& az) {
    const T r = dsqrt(x * x + y * y + z * z);
    T ux = T(0), uy = T(0), uz = T(1);
    if (r > T(0)) {
        const T ir = T(1) / r;
        ux = x * ir; uy = y * ir; uz = z * ir;
    }
    const T rc = fmin(fmax(r, mp.rmin), mp.rmax);
    const T s = (dlog(rc) - mp.lr0) * mp.idl;
    int k = int(floor(s));
    k = k < 0 ? 0 : (k > mp.nn - 2 ? mp.nn - 2 : k);
    const T t = fmin(fmax(s - T(k), T(0)), T(1));
    constexpr int nlm = kMpNlm;
    constexpr bool F4 = sizeof(TabT) == 4;
    const TabT* t0 = tab + (size_t)k * (F4 ? kMpRowF : kMpW);
    const TabT* t1 = t0 + (F4 ? kMpRowF : kMpW);
    const T irc = T(1) / rc;
    // Every gradient contribution carries the factor 1/rc, applied once at the
    // end: with P = A rc^-(l+1) + B rc^l (the term's radial factor in the
    // potential), the derivative factors A rc^-(l+2) + B rc^(l-1) are P/rc, and the
    // radial term of A r^-(l+1) is -(2l+1) A rc^-(l+2) Y_lm r^.  GX and GY hold
    // twice the x and y sums (the ladder combinations carry a factor 1/2), R the
    // radial sum.
    T U = T(0), GX = T(0), GY = T(0), GZ = T(0), R = T(0);
    T rl = T(1), rn = irc;   // rc^l, rc^-(l+1)
    T Yr[kMpL + 1], Yi[kMpL + 1], Y1r[kMpL + 1], Y1i[kMpL + 1], Y2r[kMpL + 1], Y2i[kMpL + 1];
    #pragma unroll
    for (int m = 0; m <= kMpL; ++m) { Y1r[m] = Y1i[m] = Y2r[m] = Y2i[m] = T(0); }
    // FP32: three degrees per pass, so that the three rows rotate through
    // registers instead of being copied (FP64 keeps one: its registers are full)
    constexpr int kLUnroll = sizeof(T) == 4 ? 3 : 1;
    #pragma unroll kLUnroll
    for (int l = 0; l <= kMpL; ++l) {
        // row l of Y from rows l-1 and l-2
        #pragma unroll
        for (int m = 0; m <= kMpL; ++m) {
            T yr = T(0), yi = T(0);
            if (m == l) {
                if (l == 0) {
                    yr = T(1);
                } else {
                    const T f = -mpk_o<T>(l);
                    yr = f * (ux * Y1r[m > 0 ? m - 1 : 0] - uy * Y1i[m > 0 ? m - 1 : 0]);
                    yi = f * (ux * Y1i[m > 0 ? m - 1 : 0] + uy * Y1r[m > 0 ? m - 1 : 0]);
                }
            } else if (m + 1 == l) {
                yr = mpk_o<T>(l) * uz * Y1r[m];
                yi = mpk_o<T>(l) * uz * Y1i[m];
            } else if (m + 2 <= l) {
                const T fa = mpk_a<T>(l, m), fb = mpk_b<T>(l, m);
                yr = fa * uz * Y1r[m] - fb * Y2r[m];
                yi = fa * uz * Y1i[m] - fb * Y2i[m];
            }
            Yr[m] = yr;
            Yi[m] = yi;
        }
        T Rl = T(0);
        #pragma unroll
        for (int m = 0; m <= kMpL; ++m) {
            if (m > l) break;
            const T c = mpk_c<T>(l, m);
            T Ac, Bc, As = T(0), Bs = T(0);
            if constexpr (F4) {
                // one 16-byte entry per node (the sin pair is zero for m = 0)
                const int e = 2 * l * (l + 1) + 4 * m;
                const float4 u = *reinterpret_cast<const float4*>(t0 + e);
                const float4 v = *reinterpret_cast<const float4*>(t1 + e);
                Ac = u.x + t * (v.x - u.x);
                Bc = u.y + t * (v.y - u.y);
                As = u.z + t * (v.z - u.z);
                Bs = u.w + t * (v.w - u.w);
            } else {
                const int jc = m == 0 ? (l * l) : (l * l) + 2 * m - 1;
                Ac = T(t0[jc]) + t * (T(t1[jc]) - T(t0[jc]));
                Bc = T(t0[nlm + jc]) + t * (T(t1[nlm + jc]) - T(t0[nlm + jc]));
                if (m > 0) {
                    const int js = jc + 1;
                    As = T(t0[js]) + t * (T(t1[js]) - T(t0[js]));
                    Bs = T(t0[nlm + js]) + t * (T(t1[nlm + js]) - T(t0[nlm + js]));
                }
            }
            const T yr = Yr[m], yi = Yi[m];
            const T Pc = c * (Ac * rn + Bc * rl), Ps = c * (As * rn + Bs * rl);
            U += yr * Pc + yi * Ps;
            // gradient of R_lm over r^(l-1), from row l-1 (zero for l = 0): x and y
            // from the raising and lowering combinations, z from d/dz R_lm
            const T upr = m + 1 <= kMpL ? Y1r[m + 1 <= kMpL ? m + 1 : 0] : T(0);
            const T upi = m + 1 <= kMpL ? Y1i[m + 1 <= kMpL ? m + 1 : 0] : T(0);
            if (m == 0) {
                GX += T(2) * (upr * Pc);
                GY += T(2) * (upi * Pc);
            } else {
                const T f = mpk_d<T>(l, m);
                const T dr = Y1r[m > 0 ? m - 1 : 0], di = Y1i[m > 0 ? m - 1 : 0];
                GX += (upr * Pc + upi * Ps) + f * (dr * Pc + di * Ps);
                GY += (upi * Pc - upr * Ps) - f * (di * Pc - dr * Ps);
            }
            GZ += mpk_s<T>(l, m) * (Y1r[m] * Pc + Y1i[m] * Ps);
            Rl += c * (yr * Ac + yi * As);
        }
        R += mpk_p<T>(l) * rn * Rl;
        #pragma unroll
        for (int m = 0; m <= kMpL; ++m) { Y2r[m] = Y1r[m]; Y2i[m] = Y1i[m]; Y1r[m] = Yr[m]; Y1i[m] = Yi[m]; }
        rl *= rc;
        rn *= irc;
    }
    phi = -mp.G * U;
    const T gi = mp.G * irc;
    ax = gi * (T(0.5) * GX - R * ux);
    ay = gi * (T(0.5) * GY - R * uy);
    az = gi * (GZ - R * uz);
}

// Interval of radius r: -1 below rmin, else k with r_k <= r < r_k+1 (k = nn-1 at
// and beyond rmax), decided in FP64 against the node radii.
__device__ __forceinline__ int mp_interval_f64(const double* __restrict__ rk, int nn, double lr0, double dl, double r) {
    if (r < rk[0]) return -1;
    int k = int(floor((log(r) - lr0) / dl));
    if (k > nn - 1) k = nn - 1;
    if (k < -1) k = -1;
    while (k >= 0 && r < rk[k]) --k;
    while (k + 1 <= nn - 1 && r >= rk[k + 1]) ++k;
    return k;
}

// ------------------------------------------------ update, first kick, drift
template <typename T, typename PT, int NB, uint64_t SIG>
__global__ void __launch_bounds__(sizeof(T) == 8 ? 256 : 1024) mp_kick_drift_kernel(StepArgs<T, PT> a, MpArgs<T> mp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int failed = *a.flag;
    const int J = a.lay.J, NC = a.cells.ncell;
    const int nt = blockDim.x, tid = threadIdx.x;
    // LDS: reduction scratch; the update table and the cell means are read from
    // global memory
    double* red = reinterpret_cast<double*>(smem);                        // 64

    const int t0 = ro(a.block_tile0, blockIdx.x), t1 = ro(a.block_tile0, blockIdx.x + 1);
    const uint32_t fl = a.flags;
    const uint32_t wm = (fl >> kWhatShift) & 3u;
    const bool want_cm = wm == 1 || wm == 2;
    int slot = ro(a.block_slot0, blockIdx.x) - 1, cur = -1;
    Blk<T> B{};
    Acc acc;
    if (failed) return;
    const T hdt = T(0.5) * a.dt;
    const uint32_t rb = uint32_t(a.stride * sizeof(T)), tr = uint32_t(a.stride * 2);
    for (int t = t0; t <= t1; ++t) {
        const int m = t < t1 ? ro(a.tile_model, t) : -2;
        if (m != cur) {
            if (cur >= 0) {
                wave_stats(acc.S, acc.W, acc.W2, acc.mn, red);
                __syncthreads();
                if (tid == 0) block_stats_write(red, nt >> 6, a.seg_stats + 4 * (size_t)slot);
                acc.S = acc.W = acc.W2 = 0;
                acc.mn = INFINITY;
            }
            if (m < 0) break;
            cur = m;
            ++slot;
            B.m = m;
            B.wflat = ro(a.flatw, m);
            B.cl = a.cvec + (size_t)m * J;
            B.cm = a.cellmean + (size_t)m * NC;
            B.gh = a.ghtab;
            __syncthreads();
        }
        const int64_t p0 = ro(a.tile_p0, t);
        const int cnt = ro(a.tile_cnt, t);
        for (int i = tid; i < cnt; i += nt) {
            const int64_t p = p0 + i;
            const uint32_t o = uint32_t(p) * uint32_t(sizeof(T)), ot = 7 * rb + uint32_t(p) * 2u;
            T x = ld_at<T>(a.in, o), y = ld_at<T>(a.in, o + rb), z = ld_at<T>(a.in, o + 2 * rb);
            T vx = ld_at<T>(a.in, o + 3 * rb), vy = ld_at<T>(a.in, o + 4 * rb), vz = ld_at<T>(a.in, o + 5 * rb);
            const T w = ld_at<T>(a.in, o + 6 * rb);
            uint16_t tg[kMaxBin + 1];
            #pragma unroll
            for (int b = 0; b < kMaxBin; ++b)
                tg[b] = (b < NB && b < LayoutView<SIG, T>{a.lay}.nbin()) ? ld_at<uint16_t>(a.in, ot + b * tr) : kNoBin;
            tg[kMaxBin] = want_cm ? ld_at<uint16_t>(a.in, ot + a.cellrow * tr) : 0;
            const T what_p = wm == 3 ? a.what[p] : T(1);
            const T wn = weight_update<NB, SIG>(a, B, acc, p, vy, vz, w, what_p, tg, fl);
            if (!(fl & kFrozen)) {
                // the field at x_n: stored by the previous step's second kick (or at creation)
                const T ax = ld_at<T>(mp.acc_in, o), ay = ld_at<T>(mp.acc_in, o + rb), az = ld_at<T>(mp.acc_in, o + 2 * rb);
                vx += hdt * ax; vy += hdt * ay; vz += hdt * az;
                x += a.dt * vx; y += a.dt * vy; z += a.dt * vz;
            }
            st_at(a.out, o, x);
            st_at(a.out, o + rb, y);
            st_at(a.out, o + 2 * rb, z);
            st_at(a.out, o + 3 * rb, vx);
            st_at(a.out, o + 4 * rb, vy);
            st_at(a.out, o + 5 * rb, vz);
            st_at(a.out, o + 6 * rb, wn);
        }
    }
    if (acc.bad) {
        __hip_atomic_fetch_or(a.flag, (int)acc.bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *a.bad_step = a.d_step[0];
    }
}

// ----------------------------------------------- per-interval coefficient sums
// FP64 kernels add each particle's terms to the interval sums directly (FP64
// atomics; small particle counts).
__global__ void __launch_bounds__(256) mp_coeff_atomic_kernel(MpArgs<double> mp) {
    if (*mp.flag) return;
    constexpr int nlm = kMpNlm, W = kMpW;
    const int nt = blockDim.x, tid = threadIdx.x, nn = mp.nn;
    const int t0 = ro(mp.block_tile0, blockIdx.x), t1 = ro(mp.block_tile0, blockIdx.x + 1);
    const uint32_t rb = uint32_t(mp.stride * sizeof(double));
    for (int t = t0; t < t1; ++t) {
        const int64_t p0 = ro(mp.tile_p0, t);
        const int cnt = ro(mp.tile_cnt, t);
        for (int i = tid; i < cnt; i += nt) {
            const uint32_t o = uint32_t(p0 + i) * uint32_t(sizeof(double));
            const double x = ld_at<double>(mp.src, o), y = ld_at<double>(mp.src, o + rb), z = ld_at<double>(mp.src, o + 2 * rb);
            const double mass = ld_at<double>(mp.src, o + 6 * rb) * mp.Mtot;
            const double r = sqrt(x * x + y * y + z * z);
            const int k = mp_interval_f64(mp.rk, nn, mp.lr0d, mp.dld, r);
            double ux = 0.0, uy = 0.0, uz = 1.0;
            if (r > 0.0) {
                const double ir = 1.0 / r;
                ux = x * ir; uy = y * ir; uz = z * ir;
            }
            double Yr[kMpTri], Yi[kMpTri];
            mp_harmonics(ux, uy, uz, Yr, Yi);
            double* row = mp.S + (size_t)(k + 1) * W;
            double rl = mass, rn = r > 0.0 ? mass / r : 0.0;   // m r^l, m r^-(l+1)
            const double ir = r > 0.0 ? 1.0 / r : 0.0;
            #pragma unroll
            for (int l = 0; l <= kMpL; ++l) {
                #pragma unroll
                for (int m = 0; m <= l; ++m) {
                    if (l > mp.lmax) break;   // the model's terms only (the rest stay zero)
                    const int jc = lm_at(l, m, 0);
                    atomicAdd(&row[jc], rl * Yr[tri(l, m)]);
                    atomicAdd(&row[nlm + jc], rn * Yr[tri(l, m)]);
                    if (m > 0) {
                        atomicAdd(&row[jc + 1], rl * Yi[tri(l, m)]);
                        atomicAdd(&row[nlm + jc + 1], rn * Yi[tri(l, m)]);
                    }
                }
                rl *= r;
                rn *= ir;
            }
        }
    }
}

// FP32 kernels: a counting sort of the particles by interval, then sums over
// runs of one interval in registers (no floating-point atomics; deterministic
// apart from the order within an (interval, block) pair, which the scatter's
// integer atomics decide).

// Interval of a particle at FP32 (x, y, z): the FP32 decision unless r lies
// within 1e-4 of an interval of a node radius (or of rmin), else the FP64 one.
__device__ __forceinline__ int mp_interval_f32(const MpArgs<float>& mp, float x, float y, float z) {
    const float r = sqrtf(x * x + y * y + z * z);
    const float s = (__logf(r) - mp.lr0) * mp.idl;
    const float fr = s - floorf(s);
    if (!(r > 0.0f) || fr < 1e-4f || fr > 1.0f - 1e-4f || fabsf(r - mp.rmin) < 1e-4f * mp.rmin) {
        const double rd = sqrt(double(x) * double(x) + double(y) * double(y) + double(z) * double(z));
        return mp_interval_f64(mp.rk, mp.nn, mp.lr0d, mp.dld, rd);
    }
    return r < mp.rmin ? -1 : max(-1, min(int(floorf(s)), mp.nn - 1));
}

// Exclusive scan of v over the 64 lanes of a wave; *total gets the sum.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total) {
    const int lane = threadIdx.x & 63;
    uint32_t inc = v;
    #pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
    }
    *total = __shfl(inc, 63, 64);
    return inc - v;
}

// Block b's particles [b R, (b + 1) R): interval keys and per-interval counts.
constexpr int kMpSortRun = 8;   // particles per thread per round of the sort kernels

__global__ void __launch_bounds__(kMpSortThreads) mp_interval_kernel(MpArgs<float> mp) {
    __shared__ uint32_t cnt[kMpMaxNodes + 1];
    if (*mp.flag) return;
    const int nt = blockDim.x, tid = threadIdx.x, b = blockIdx.x, nn = mp.nn;
    for (int i = tid; i <= nn; i += nt) cnt[i] = 0u;
    __syncthreads();
    const int64_t p0 = (int64_t)b * mp.R, p1 = min(mp.n, p0 + mp.R);
    const uint32_t rb = uint32_t(mp.stride * 4);
    // kMpSortRun particles per thread per round, all loaded before the first is
    // decided (indexes past the end re-read the last particle, rewrite its key
    // and count nothing)
    for (int64_t pb = p0 + tid; pb < p1; pb += (int64_t)kMpSortRun * nt) {
        float x[kMpSortRun], y[kMpSortRun], z[kMpSortRun];
        #pragma unroll
        for (int u = 0; u < kMpSortRun; ++u) {
            const uint32_t o = uint32_t(min(pb + (int64_t)u * nt, p1 - 1)) * 4u;
            x[u] = ld_at<float>(mp.src, o);
            y[u] = ld_at<float>(mp.src, o + rb);
            z[u] = ld_at<float>(mp.src, o + 2 * rb);
        }
        #pragma unroll
        for (int u = 0; u < kMpSortRun; ++u) {
            const int64_t p = pb + (int64_t)u * nt;
            const int k1 = mp_interval_f32(mp, x[u], y[u], z[u]) + 1;
            mp.key[min(p, p1 - 1)] = (uint16_t)k1;
            atomicAdd(&cnt[k1], p < p1 ? 1u : 0u);
        }
    }
    __syncthreads();
    for (int i = tid; i <= nn; i += nt) mp.counts[(size_t)i * mp.G_sort + b] = cnt[i];
}

// Interval k: first position of each block's particles within the interval
// (exclusive scan over the blocks in order) and the interval's total.
__global__ void __launch_bounds__(256) mp_offsets_kernel(MpArgs<float> mp) {
    __shared__ uint32_t wsum[4];
    if (*mp.flag) return;
    const int k = blockIdx.x, tid = threadIdx.x, G = mp.G_sort;
    const uint32_t* src = mp.counts + (size_t)k * G;
    uint32_t c[4], sum = 0;
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int b = tid * 4 + j;
        c[j] = b < G ? src[b] : 0u;
        sum += c[j];
    }
    uint32_t wtot;
    const uint32_t excl = wave_excl_scan(sum, &wtot);
    if ((tid & 63) == 0) wsum[tid >> 6] = wtot;
    __syncthreads();
    uint32_t run = excl;
    for (int w = 0; w < (tid >> 6); ++w) run += wsum[w];
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int b = tid * 4 + j;
        if (b < G) mp.offs[(size_t)k * G + b] = run;
        run += c[j];
    }
    if (tid == 255) mp.total[k] = run;
}

// Scatter (x, y, z, w) of block b's particles to their sorted positions.
__global__ void __launch_bounds__(kMpSortThreads) mp_scatter_kernel(MpArgs<float> mp) {
    __shared__ uint32_t off[kMpMaxNodes + 1];
    if (*mp.flag) return;
    const int nt = blockDim.x, tid = threadIdx.x, b = blockIdx.x, nn = mp.nn;
    if (tid < 64) {
        // first position of interval k = sum of the totals below it
        uint32_t run = 0;
        for (int k0 = 0; k0 <= nn; k0 += 64) {
            const int k = k0 + tid;
            const uint32_t t = k <= nn ? mp.total[k] : 0u;
            uint32_t tot;
            const uint32_t ex = wave_excl_scan(t, &tot);
            if (k <= nn) off[k] = run + ex + mp.offs[(size_t)k * mp.G_sort + b];
            run += tot;
        }
    }
    __syncthreads();
    const int64_t p0 = (int64_t)b * mp.R, p1 = min(mp.n, p0 + mp.R);
    const uint32_t rb = uint32_t(mp.stride * 4);
    // kMpSortRun particles per thread per round, all loaded before the first
    // position is claimed (indexes past the end re-read the last particle and
    // claim nothing)
    for (int64_t pb = p0 + tid; pb < p1; pb += (int64_t)kMpSortRun * nt) {
        float4 v[kMpSortRun];
        uint32_t key[kMpSortRun];
        #pragma unroll
        for (int u = 0; u < kMpSortRun; ++u) {
            const int64_t p = min(pb + (int64_t)u * nt, p1 - 1);
            const uint32_t o = uint32_t(p) * 4u;
            v[u] = make_float4(ld_at<float>(mp.src, o), ld_at<float>(mp.src, o + rb), ld_at<float>(mp.src, o + 2 * rb),
                               ld_at<float>(mp.src, o + 6 * rb));
            key[u] = mp.key[p];
        }
        #pragma unroll
        for (int u = 0; u < kMpSortRun; ++u) {
            if (pb + (int64_t)u * nt < p1) {
                const uint32_t pos = atomicAdd(&off[key[u]], 1u);
                mp.sorted[pos] = v[u];
            }
        }
    }
}

// First sorted position (base) and first chunk (c0) of every interval k = 0..nn+1,
// into LDS (wave 0 of the block; the caller synchronises).
__device__ __forceinline__ void mp_chunk_table(const MpArgs<float>& mp, uint32_t* base, uint32_t* c0) {
    const int tid = threadIdx.x, nn = mp.nn;
    if (tid >= 64) return;
    uint32_t rb = 0, rc = 0;
    for (int k0 = 0; k0 <= nn + 1; k0 += 64) {
        const int k = k0 + tid;
        const uint32_t t = k <= nn ? mp.total[k] : 0u;
        const uint32_t nc = (t + kMpChunk - 1) / kMpChunk;
        uint32_t tb, tc;
        const uint32_t eb = wave_excl_scan(t, &tb), ec = wave_excl_scan(nc, &tc);
        if (k <= nn + 1) { base[k] = rb + eb; c0[k] = rc + ec; }
        rb += tb;
        rc += tc;
    }
}

// One wave per chunk (up to kMpChunk sorted particles of one interval): each lane
// sums the terms of its particles in registers, the wave adds its lanes, and the
// chunk's 162 sums go to its own partial row.
__global__ void __launch_bounds__(256) mp_accum_kernel(MpArgs<float> mp) {
    __shared__ uint32_t base[kMpMaxNodes + 2], c0[kMpMaxNodes + 2];
    if (*mp.flag) return;
    mp_chunk_table(mp, base, c0);
    __syncthreads();
    const int nn = mp.nn, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= (int)c0[nn + 1]) return;
    // interval of chunk c: the last k with c0[k] <= c (intervals without chunks
    // share c0 with the next one)
    int lo = 0, hi = nn;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int)c0[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t start = base[lo] + uint32_t(c - (int)c0[lo]) * kMpChunk;
    const int cnt = (int)min((uint32_t)kMpChunk, base[lo + 1] - start);
    const float Mtot = mp.Mtot;
    float acc[kMpW];
    #pragma unroll
    for (int v = 0; v < kMpW; ++v) acc[v] = 0.0f;
    float4 nxt = mp.sorted[start + min(lane, cnt - 1)];
    #pragma unroll 1
    for (int i = 0; i < kMpLaneRun; ++i) {
        const int q = lane + 64 * i;
        const float4 cur = nxt;
        if (i + 1 < kMpLaneRun) nxt = mp.sorted[start + min(q + 64, cnt - 1)];
        // lanes past the chunk's end re-read its last particle with zero mass
        const float x = cur.x, y = cur.y, z = cur.z, mass = q < cnt ? cur.w * Mtot : 0.0f;
        const float r = sqrtf(x * x + y * y + z * z);
        float ux = 0.0f, uy = 0.0f, uz = 1.0f, ir = 0.0f;
        if (r > 0.0f) {
            ir = 1.0f / r;
            ux = x * ir; uy = y * ir; uz = z * ir;
        }
        float rl = mass, rn = mass * ir;   // m r^l, m r^-(l+1)
        float Y1r[kMpL + 1], Y1i[kMpL + 1], Y2r[kMpL + 1], Y2i[kMpL + 1];
        #pragma unroll
        for (int m = 0; m <= kMpL; ++m) Y1r[m] = Y1i[m] = Y2r[m] = Y2i[m] = 0.0f;
        #pragma unroll
        for (int l = 0; l <= kMpL; ++l) {
            float Yr[kMpL + 1], Yi[kMpL + 1];
            #pragma unroll
            for (int m = 0; m <= l; ++m) {
                if (m == l) {
                    if (l == 0) { Yr[0] = 1.0f; Yi[0] = 0.0f; }
                    else {
                        const float f = -float(2 * l - 1);
                        const int mp1 = m > 0 ? m - 1 : 0;
                        Yr[m] = f * (ux * Y1r[mp1] - uy * Y1i[mp1]);
                        Yi[m] = f * (ux * Y1i[mp1] + uy * Y1r[mp1]);
                    }
                } else if (m + 1 == l) {
                    Yr[m] = float(2 * l - 1) * uz * Y1r[m];
                    Yi[m] = float(2 * l - 1) * uz * Y1i[m];
                } else {
                    const float fa = float(2 * l - 1) / float(l - m), fb = float(l + m - 1) / float(l - m);
                    Yr[m] = fa * uz * Y1r[m] - fb * Y2r[m];
                    Yi[m] = fa * uz * Y1i[m] - fb * Y2i[m];
                }
                const int jc = lm_at(l, m, 0);
                acc[jc] += rl * Yr[m];
                acc[kMpNlm + jc] += rn * Yr[m];
                if (m > 0) {
                    acc[jc + 1] += rl * Yi[m];
                    acc[kMpNlm + jc + 1] += rn * Yi[m];
                }
            }
            #pragma unroll
            for (int m = 0; m <= l; ++m) {
                if (l >= 1 && m <= l - 1) { Y2r[m] = Y1r[m]; Y2i[m] = Y1i[m]; }
                Y1r[m] = Yr[m];
                Y1i[m] = Yi[m];
            }
            rl *= r;
            rn *= ir;
        }
    }
    // Wave sums of the kMpW values, reduced and scattered at once: padded to 3 x
    // 64 values, each level pairs lanes L and L ^ o; a lane keeps the half of its
    // values that its bit o selects, sends the other half to its partner and adds
    // what it receives.  After the six levels lane L holds the sums of values
    // 3L, 3L + 1 and 3L + 2 (189 independent exchanges instead of 6 dependent
    // ones per value).
    constexpr int kRs = 3 * 64;
    static_assert(kMpW <= kRs, "reduce-scatter holds 3 values per lane");
    float a[kRs];
    #pragma unroll
    for (int v = 0; v < kRs; ++v) a[v] = v < kMpW ? acc[v] : 0.0f;
    #pragma unroll
    for (int lv = 0; lv < 6; ++lv) {
        const int o = 32 >> lv, h = (kRs / 2) >> lv;
        const bool up = (lane & o) != 0;
        #pragma unroll
        for (int i = 0; i < h; ++i) {
            const float keep = up ? a[i + h] : a[i];
            const float send = up ? a[i] : a[i + h];
            a[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    float* dst = mp.part + (size_t)c * kMpW;
    #pragma unroll
    for (int j = 0; j < 3; ++j)
        if (3 * lane + j < kMpW) dst[3 * lane + j] = a[j];
}

// Interval sums of key k (interval k - 1, row k of S): the key's chunks added in
// chunk order in FP64; terms above the model's lmax are zero.
__global__ void __launch_bounds__(256) mp_chunksum_kernel(MpArgs<float> mp) {
    __shared__ uint32_t base[kMpMaxNodes + 2], c0[kMpMaxNodes + 2];
    if (*mp.flag) return;
    mp_chunk_table(mp, base, c0);
    __syncthreads();
    const int k = blockIdx.x, v = threadIdx.x;
    if (v >= kMpW) return;
    const int j0 = (int)c0[k], j1 = (int)c0[k + 1];
    const float* src = mp.part + v;
    double acc = 0.0;
    // 32 chunk rows in flight per round, added in chunk order
    constexpr int kRun = 32;
    for (int j = j0; j < j1; j += kRun) {
        float u[kRun];
        #pragma unroll
        for (int q = 0; q < kRun; ++q) u[q] = src[(size_t)min(j + q, j1 - 1) * kMpW];
        #pragma unroll
        for (int q = 0; q < kRun; ++q) acc += j + q < j1 ? double(u[q]) : 0.0;
    }
    const int jj = v < kMpNlm ? v : v - kMpNlm;
    int l = 0;
    while ((l + 1) * (l + 1) <= jj) ++l;
    mp.S[(size_t)k * kMpW + v] = l <= mp.lmax ? acc : 0.0;
}

// Node coefficients of column v (one block each): A(r_k) = sum of the intervals
// below r_k (prefix scan), B(r_k) = sum of the intervals from r_k up (suffix
// scan), in FP64 in node order.  The FP64 kernels' interval sums are cleared for
// the next build.
template <typename T>
__global__ void __launch_bounds__(128) mp_scan_kernel(MpArgs<T> mp) {
    __shared__ double colA[kMpMaxNodes + 1], colB[kMpMaxNodes + 1];
    if (*mp.flag) return;
    const int v = blockIdx.x, nn = mp.nn, nlm = mp.nlm, tid = threadIdx.x;
    constexpr int W = kMpW;
    for (int k = tid; k <= nn; k += blockDim.x) {
        colA[k] = mp.S[(size_t)k * W + v];
        colB[k] = mp.S[(size_t)k * W + kMpNlm + v];
    }
    __syncthreads();
    // place of coefficient v (A; B one further) in a node's FP32 entries
    int l = 0;
    while ((l + 1) * (l + 1) <= v) ++l;
    const int m = (v - l * l + 1) >> 1, sn = v > l * l && ((v - l * l) & 1) == 0;
    const int e = 2 * l * (l + 1) + 4 * m + 2 * sn;
    constexpr bool F4 = sizeof(T) == 4;
    const int rowlen = F4 ? kMpRowF : W, ea = F4 ? e : v, eb = F4 ? e + 1 : kMpNlm + v;
    // wave 0: A at node k = colA[0] + ... + colA[k]; wave 1: B at node k =
    // colB[nn] + ... + colB[k + 1], i.e. the same scan along i = nn - 1 - k.
    // Each lane adds a run of kRun consecutive terms in order; the runs' totals
    // are scanned across the wave, and each lane adds the total before its run
    // to its own partial sums (a fixed order).
    const int lane = tid & 63, wv = tid >> 6;
    if (wv < 2) {
        constexpr int kRun = (kMpMaxNodes + 63) / 64;
        const int i0 = lane * kRun;
        double part[kRun], run = 0.0;
        #pragma unroll
        for (int q = 0; q < kRun; ++q) {
            const int i = i0 + q;
            run += i < nn ? (wv == 0 ? colA[i] : colB[nn - i]) : 0.0;
            part[q] = run;
        }
        double inc = run;
        #pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double u = __shfl_up(inc, d, 64);
            if (lane >= d) inc += u;
        }
        double before = __shfl_up(inc, 1, 64);
        if (lane == 0) before = 0.0;
        #pragma unroll
        for (int q = 0; q < kRun; ++q) {
            const int i = i0 + q;
            if (i < nn) {
                const double val = before + part[q];
                const int k = wv == 0 ? i : nn - 1 - i;
                if (v < nlm) (wv == 0 ? mp.A64 : mp.B64)[(size_t)k * nlm + v] = val;
                mp.tab_out[(size_t)k * rowlen + (wv == 0 ? ea : eb)] = T(val);
            }
        }
    }
    if constexpr (sizeof(T) == 8) {
        for (int k = tid; k <= nn; k += blockDim.x) {
            mp.S[(size_t)k * W + v] = 0.0;
            mp.S[(size_t)k * W + kMpNlm + v] = 0.0;
        }
    }
}

// -------------------------------------------------------------- second kick
template <typename T>
__global__ void __launch_bounds__(sizeof(T) == 8 ? 256 : 1024) mp_kick_kernel(MpArgs<T> mp) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool F32 = sizeof(T) == 4;
    const int failed = *mp.flag;
    const int nt = blockDim.x, tid = threadIdx.x;
    float* tabl = reinterpret_cast<float*>(smem);
    const int NT = F32 ? mp.nn * kMpRowF : 0;
    if constexpr (F32)
        mp_table_to_lds(reinterpret_cast<float4*>(tabl), reinterpret_cast<const float4*>(mp.tab), NT / 4, tid, nt);
    __syncthreads();
    if (failed) return;
    const int t0 = ro(mp.block_tile0, blockIdx.x), t1 = ro(mp.block_tile0, blockIdx.x + 1);
    const uint32_t rb = uint32_t(mp.stride * sizeof(T));
    T* dst = const_cast<T*>(mp.src);
    for (int t = t0; t < t1; ++t) {
        const int64_t p0 = ro(mp.tile_p0, t);
        const int cnt = ro(mp.tile_cnt, t);
        for (int i = tid; i < cnt; i += nt) {
            const uint32_t o = uint32_t(p0 + i) * uint32_t(sizeof(T));
            const T x = ld_at<T>(mp.src, o), y = ld_at<T>(mp.src, o + rb), z = ld_at<T>(mp.src, o + 2 * rb);
            T phi, ax, ay, az;
            if constexpr (F32) mp_field<T, float>(mp, tabl, x, y, z, phi, ax, ay, az);
            else mp_field<T, T>(mp, mp.tab, x, y, z, phi, ax, ay, az);
            st_at(mp.acc_out, o, ax);
            st_at(mp.acc_out, o + rb, ay);
            st_at(mp.acc_out, o + 2 * rb, az);
            if (mp.kick == 1) {
                st_at(dst, o + 3 * rb, ld_at<T>(mp.src, o + 3 * rb) + mp.hdt * ax);
                st_at(dst, o + 4 * rb, ld_at<T>(mp.src, o + 4 * rb) + mp.hdt * ay);
                st_at(dst, o + 5 * rb, ld_at<T>(mp.src, o + 5 * rb) + mp.hdt * az);
            }
        }
    }
}

// ------------------------------------------------------------------ launchers
template <typename T, typename PT, int NB, uint64_t SIG>
static hipError_t launch_kd(const StepArgs<T, PT>& a, const MpArgs<T>& mp, int blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((mp_kick_drift_kernel<T, PT, NB, SIG>), dim3(blocks), dim3(sizeof(T) == 8 ? 256 : 1024), lds, s,
                       a, mp);
    return hipGetLastError();
}

template <typename T, typename PT>
hipError_t launch_mp_step(const StepArgs<T, PT>& a, const MpArgs<T>& mp, uint64_t sig, int nbin, int blocks,
                          const MpLds& lds, hipStream_t s) {
    // the sky pixels + kinematics + shells layout has a kernel of its own (kinds
    // and moments fixed at compile time), as in the fused step kernel
    if constexpr (sizeof(T) == 4)
        if (sig == kSigPixKinShell) return launch_kd<T, PT, 4, kSigPixKinShell>(a, mp, blocks, lds.kick_drift, s);
    if (nbin <= 2) return launch_kd<T, PT, 2, 0>(a, mp, blocks, lds.kick_drift, s);
    return launch_kd<T, PT, 4, 0>(a, mp, blocks, lds.kick_drift, s);
}

template <typename T>
hipError_t launch_mp_build(const MpArgs<T>& mp, int blocks, const MpLds& lds, hipStream_t s, hipEvent_t ek0,
                           hipEvent_t ek1) {
    hipError_t e;
    if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL(mp_interval_kernel, dim3(mp.G_sort), dim3(kMpSortThreads), 0, s, mp);
        hipLaunchKernelGGL(mp_offsets_kernel, dim3(mp.nn + 1), dim3(256), 0, s, mp);
        hipLaunchKernelGGL(mp_scatter_kernel, dim3(mp.G_sort), dim3(kMpSortThreads), 0, s, mp);
        hipLaunchKernelGGL(mp_accum_kernel, dim3((mp.maxchunk + 3) / 4), dim3(256), 0, s, mp);
        hipLaunchKernelGGL(mp_chunksum_kernel, dim3(mp.nn + 1), dim3(256), 0, s, mp);
    } else {
        hipLaunchKernelGGL(mp_coeff_atomic_kernel, dim3(blocks), dim3(256), 0, s, mp);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((mp_scan_kernel<T>), dim3(kMpNlm), dim3(128), 0, s, mp);
    if ((e = hipGetLastError()) != hipSuccess || !mp.kick) return e;
    if (ek0 || ek1)   // (timing: the events take the kick's own start and end times)
        hipExtLaunchKernelGGL((mp_kick_kernel<T>), dim3(blocks), dim3(sizeof(T) == 8 ? 256 : 1024),
                              (uint32_t)lds.kick, s, ek0, ek1, 0u, mp);
    else
        hipLaunchKernelGGL((mp_kick_kernel<T>), dim3(blocks), dim3(sizeof(T) == 8 ? 256 : 1024), lds.kick, s, mp);
    return hipGetLastError();
}

template <typename T, typename PT>
hipError_t set_mp_lds_limit(size_t lds) {
    for (const void* f : {(const void*)mp_kick_drift_kernel<T, PT, 2, 0>, (const void*)mp_kick_drift_kernel<T, PT, 4, 0>,
                          (const void*)mp_kick_kernel<T>}) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if constexpr (sizeof(T) == 4)
        return hipFuncSetAttribute((const void*)mp_kick_drift_kernel<T, PT, 4, kSigPixKinShell>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

template hipError_t launch_mp_step<float, float>(const StepArgs<float, float>&, const MpArgs<float>&, uint64_t, int, int,
                                                 const MpLds&, hipStream_t);
template hipError_t launch_mp_step<double, double>(const StepArgs<double, double>&, const MpArgs<double>&, uint64_t,
                                                   int, int, const MpLds&, hipStream_t);
template hipError_t launch_mp_build<float>(const MpArgs<float>&, int, const MpLds&, hipStream_t, hipEvent_t,
                                          hipEvent_t);
template hipError_t launch_mp_build<double>(const MpArgs<double>&, int, const MpLds&, hipStream_t, hipEvent_t,
                                           hipEvent_t);
template hipError_t set_mp_lds_limit<float, float>(size_t);
template hipError_t set_mp_lds_limit<double, double>(size_t);

}  // namespace m2m
