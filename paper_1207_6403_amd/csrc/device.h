// device.h -- per-particle device functions of the M2M step (gfx950, wave64).
//
// Everything here is evaluated in registers for one particle: the potential
// and acceleration (section 2: a potential fixed and known a priori), the
// observation bins of the layout (section 2: observables compared with the
// target; section 1: photometry and line-of-sight kinematics) and the
// phase-space cell of the moving prior (section 2.1: integrals of motion E, L,
// Lz).  Kernels include this header; the host never calls these functions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace m2m {

constexpr int kMaxBin = 4;
constexpr int kMaxEntries = 3 * kMaxBin;   // non-zero K_j per particle

// Potential parameters in the particle precision, with derived constants.
template <typename T>
struct Pot {
    int32_t kind;       // M2M_POT_*
    int32_t lc_off;     // offset of this model's Ec table (Hernquist+NFW Lc(E))
    T GM, a;            // Hernquist
    T v2, Rc2, iq2;     // logarithmic: v0^2, Rc^2, 1/q^2
    T GMh, rs, irs;     // NFW halo
};

// Observation layout in the particle precision.  Edges live in LDS.
template <typename T>
struct Layout {
    T cosi, sini;
    int32_t nbin;
    int32_t J;
    int32_t kind[kMaxBin];
    int32_t nmom[kMaxBin];
    int32_t mom[kMaxBin][3];
    int32_t off[kMaxBin];      // first observable index of the binning
    int32_t nb[kMaxBin];       // bins per moment
    int32_t edge0[kMaxBin];    // offset of the binning's edges in the edge table
    int32_t nx[kMaxBin], ny[kMaxBin];
    T x0[kMaxBin], wx[kMaxBin], y0[kMaxBin], wy[kMaxBin];
};

// Moving-prior cell geometry.
template <typename T>
struct Cells {
    int32_t n0, n1, n2;   // cells along E, L/Lc or Lz/Lc, Lz/L
    int32_t ax2;          // 0: L/Lc in [0,1]; 1: Lz/Lc in [-1,1]
    int32_t ncell;
};

// ------------------------------------------------------------------ potentials
template <typename T> __device__ __forceinline__ T dsqrt(T v) { return sqrt(v); }
template <typename T> __device__ __forceinline__ T dlog(T v) { return log(v); }
template <typename T> __device__ __forceinline__ T dexp(T v) { return exp(v); }
template <typename T> __device__ __forceinline__ T dlog1p(T v) { return log1p(v); }

// Phi(x) and a = -grad Phi.  POT is the compile-time potential kind.
template <int POT, typename T>
__device__ __forceinline__ void potential(const Pot<T>& p, T x, T y, T z, T& phi, T& ax, T& ay, T& az) {
    if (POT == 1) {   // logarithmic
        T s = p.Rc2 + x * x + y * y + z * z * p.iq2;
        T f = p.v2 / s;
        phi = T(0.5) * p.v2 * dlog(s);
        ax = -f * x;
        ay = -f * y;
        az = -f * z * p.iq2;
        return;
    }
    T r2 = x * x + y * y + z * z;
    T r = dsqrt(r2);
    T u = r + p.a;
    T ph = -p.GM / u;
    T g_over_r = r > T(0) ? p.GM / (u * u * r) : T(0);   // (dPhi/dr)/r
    if (POT == 2 && p.GMh > T(0)) {
        T xx = r * p.irs;
        T l1 = dlog1p(xx);
        ph += r > T(0) ? -p.GMh * l1 / r : -p.GMh * p.irs;
        // dPhi_NFW/dr = G Mh/rs^2 * f(x), f = ln(1+x)/x^2 - 1/(x(1+x));
        // near x = 0 the two terms cancel, so a series is used there.
        T f;
        if (xx < T(0.05)) {
            f = T(0.5) + xx * (T(-2.0 / 3.0) + xx * (T(0.75) + xx * (T(-0.8) + xx * (T(5.0 / 6.0) - xx * T(6.0 / 7.0)))));
        } else {
            f = l1 / (xx * xx) - T(1) / (xx * (T(1) + xx));
        }
        g_over_r += r > T(0) ? p.GMh * p.irs * p.irs * f / r : T(0);
    }
    phi = ph;
    ax = -g_over_r * x;
    ay = -g_over_r * y;
    az = -g_over_r * z;
}

// dPhi/dr and d2Phi/dr2 of the spherical kinds (Hernquist + NFW Lc(E) Newton).
template <typename T>
__device__ __forceinline__ void radial_derivs(const Pot<T>& p, T r, T& phi, T& d1, T& d2) {
    T u = r + p.a;
    phi = -p.GM / u;
    d1 = p.GM / (u * u);
    d2 = T(-2) * p.GM / (u * u * u);
    if (p.GMh > T(0)) {
        T xx = r * p.irs;
        T l1 = dlog1p(xx);
        T rrs = r + p.rs;
        phi += -p.GMh * l1 / r;
        d1 += p.GMh * (l1 / (r * r) - T(1) / (r * rrs));
        d2 += p.GMh * (T(1) / (r * r * rrs) + (T(2) * r + p.rs) / (r * r * rrs * rrs) - T(2) * l1 / (r * r * r));
    }
}

// Angular momentum of the circular orbit of energy E.  Returns a value <= 0 to
// mean "infinite" (E at or above the top of the potential) and a negative
// sentinel below the bottom is not needed: the ratio is clamped by the caller.
template <int POT, typename T>
__device__ __forceinline__ T circular_L(const Pot<T>& p, const T* __restrict__ ectab, T E) {
    if (POT == 0) {
        // 2E u^2 + GM u + GM a = 0 with u = r_c + a; the stable form
        // r_c = 4a(GM + E a)/(sqrt(GM^2 - 8 E GM a) - GM - 4 E a).
        T D = p.GM * p.GM - T(8) * E * p.GM * p.a;
        if (!(E < T(0))) return T(-1);
        T rc = T(4) * p.a * (p.GM + E * p.a) / (dsqrt(D) - p.GM - T(4) * E * p.a);
        if (!(rc > T(0))) return T(0);
        return rc * dsqrt(p.GM * rc) / (rc + p.a);
    } else if (POT == 1) {
        // E = v0^2/2 [1 - Rc^2/s + ln s], s = Rc^2 + R^2: solve t = ln s of
        // t - Rc^2 e^-t = k (increasing, concave) by Newton from the left.
        T k = T(2) * E / p.v2 - T(1);
        T tmin = dlog(p.Rc2);
        T t = k > tmin ? k : tmin;
        #pragma unroll
        for (int it = 0; it < 8; ++it) {
            T e = p.Rc2 * dexp(-t);
            t = t - (t - e - k) / (T(1) + e);
        }
        T s = dexp(t);
        T R2 = s - p.Rc2;
        if (!(R2 > T(0))) return T(0);
        return dsqrt(p.v2) * R2 / dsqrt(s);
    } else {
        // Hernquist + NFW: bracket ln r in the model's table of E_c(r) at 128
        // log-spaced radii on [1e-4, 1e4] (r_k = 1e-4 * 10^(8k/127)), then Newton
        // on E_c(r) = Phi + r Phi'/2 with dE_c/dr = (3 Phi' + r Phi'')/2.
        const T* tab = ectab + p.lc_off;
        if (E <= tab[0] || E >= tab[127]) {
            T rr = E <= tab[0] ? T(1e-4) : T(1e4);
            T ph, d1, d2;
            radial_derivs(p, rr, ph, d1, d2);
            return rr * dsqrt(rr * d1);
        }
        int lo = 0, hi = 127;
        #pragma unroll
        for (int it = 0; it < 7; ++it) {
            int mid = (lo + hi) >> 1;
            if (tab[mid] <= E) lo = mid; else hi = mid;
        }
        const T dl = T(8.0 * 2.302585092994046 / 127.0);
        T t = (E - tab[lo]) / (tab[hi] - tab[lo]);
        T lr = T(-4.0 * 2.302585092994046) + (T(lo) + t) * dl;
        T r = dexp(lr);
        #pragma unroll
        for (int it = 0; it < 3; ++it) {
            T ph, d1, d2;
            radial_derivs(p, r, ph, d1, d2);
            T Ec = ph + T(0.5) * r * d1;
            T dE = T(0.5) * (T(3) * d1 + r * d2);
            r = r - (Ec - E) / dE;
        }
        T ph, d1, d2;
        radial_derivs(p, r, ph, d1, d2);
        return r * dsqrt(r * d1);
    }
}

__device__ __forceinline__ int clamp_cell(float f, int n) {
    if (!(f >= 0.0f)) return 0;
    if (f >= float(n)) return n - 1;
    return int(f);
}
__device__ __forceinline__ int clamp_cell(double f, int n) {
    if (!(f >= 0.0)) return 0;
    if (f >= double(n)) return n - 1;
    return int(f);
}

// Cell of the moving prior for a particle of energy E.
template <int POT, typename T>
__device__ __forceinline__ int prior_cell(const Pot<T>& p, const T* __restrict__ ectab, const Cells<T>& c,
                                          T Emin, T Ewid, T E, T x, T y, T z, T vx, T vy, T vz) {
    T Lx = y * vz - z * vy, Ly = z * vx - x * vz, Lz = x * vy - y * vx;
    T L = dsqrt(Lx * Lx + Ly * Ly + Lz * Lz);
    T Lc = circular_L<POT, T>(p, ectab, E);
    int iE = clamp_cell((E - Emin) / Ewid * T(c.n0), c.n0);
    int i2;
    if (c.ax2 == 0) {
        T f = Lc > T(0) ? L / Lc : (Lc < T(0) ? T(0) : T(1e30));
        i2 = clamp_cell(f * T(c.n1), c.n1);
    } else {
        T f = Lc > T(0) ? Lz / Lc : (Lc < T(0) ? T(0) : (Lz > T(0) ? T(1e30) : T(-1e30)));
        i2 = clamp_cell((f + T(1)) * T(0.5) * T(c.n1), c.n1);
    }
    int i3 = 0;
    if (c.n2 > 1) {
        T f = L > T(0) ? Lz / L : T(0);
        i3 = clamp_cell((f + T(1)) * T(0.5) * T(c.n2), c.n2);
    }
    return (iE * c.n1 + i2) * c.n2 + i3;
}

// ---------------------------------------------------------------- observables
// Bin of value v against nedge increasing edges in LDS: -1 outside [e0, e_last).
template <typename T>
__device__ __forceinline__ int edge_bin(const T* __restrict__ e, int ne, T v) {
    if (!(v >= e[0]) || !(v < e[ne - 1])) return -1;
    int lo = 0, hi = ne - 1;   // e[lo] <= v < e[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (v >= e[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

// Kernel entries K_j of one phase-space point in fixed slots e = 3 b + m
// (binning b, m-th listed moment); jj[e] = -1 marks an empty slot.  Fixed
// slots keep both arrays in registers (every index is a compile-time constant
// once the loops are unrolled).
template <typename T>
__device__ __forceinline__ void kernel_entries(const Layout<T>& L, const T* __restrict__ edges,
                                               T x, T y, T z, T vy, T vz, int (&jj)[kMaxEntries],
                                               T (&K)[kMaxEntries]) {
    const T X = x;
    const T Ys = y * L.cosi - z * L.sini;
    const T vl = vy * L.sini + vz * L.cosi;
    #pragma unroll
    for (int b = 0; b < kMaxBin; ++b) {
        int k = -1;
        if (b < L.nbin) {
            if (L.kind[b] == 3) {
                const T fx = floor((X - L.x0[b]) / L.wx[b] * T(L.nx[b]));
                const T fy = floor((Ys - L.y0[b]) / L.wy[b] * T(L.ny[b]));
                if (fx >= T(0) && fx < T(L.nx[b]) && fy >= T(0) && fy < T(L.ny[b]))
                    k = int(fy) * L.nx[b] + int(fx);
            } else {
                const T rad = L.kind[b] == 1 ? dsqrt(x * x + y * y + z * z) : dsqrt(X * X + Ys * Ys);
                k = edge_bin(edges + L.edge0[b], L.nb[b] + 1, rad);
            }
        }
        #pragma unroll
        for (int m = 0; m < 3; ++m) {
            const bool on = k >= 0 && m < L.nmom[b];
            const int mo = L.mom[b][m];
            jj[3 * b + m] = on ? L.off[b] + m * L.nb[b] + k : -1;
            K[3 * b + m] = mo == 0 ? T(1) : (mo == 1 ? vl : vl * vl);
        }
    }
}

}  // namespace m2m
