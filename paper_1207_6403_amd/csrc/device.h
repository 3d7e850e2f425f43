// device.h -- per-particle device functions of the M2M step (gfx950, wave64).
//
// Everything here is evaluated in registers for one particle: the potential
// and acceleration (section 2: a potential fixed and known a priori), the
// observation bins of the layout (section 2: observables compared with the
// target; section 1: photometry and line-of-sight kinematics) and the
// phase-space cell of the moving prior (section 2.1: integrals of motion E, L,
// Lz).  Kernels include this header; the host never calls these functions.
//
// Integer decisions (which bin, which prior cell) are taken in FP64.  The FP32
// kernels first decide in FP32 and keep that answer when the fractional bin
// coordinate is further than a guard band from every edge (the FP32 error is
// an order of magnitude below the band); a decision inside the band -- a few in
// ten thousand -- is re-taken from the same coordinates in FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace m2m {

constexpr int kMaxBin = 4;
constexpr int kMaxEntries = 3 * kMaxBin;   // kernel entries K_j per particle (fixed slots)
constexpr int kLcTab = 256;                // circular-orbit energies per model (FP64 path)
constexpr int kLcE = 2048;                 // uniform-E Lc(E) table per model (FP32 path)
constexpr float kGuardCell = 1e-4f;        // guard band, in cells, of the FP32 prior coordinates
// Guard bands of the FP32 bin decisions: twice a bound on the difference between
// the FP32 coordinate and the FP64 one computed from the same FP32 particle (u =
// 2^-24, the FP32 unit roundoff), plus a floor that keeps a coordinate exactly
// on an edge open.
constexpr float kU32 = 5.9604645e-8f;
constexpr float kGuardBinFloor = 1e-6f;    // bins

// Potential parameters with derived constants.
template <typename T>
struct Pot {
    int32_t kind;       // M2M_POT_*
    int32_t lc_off;     // this model's offset in the circular-orbit table
    T GM, a;            // Hernquist
    T v2, Rc2, iq2;     // logarithmic: v0^2, Rc^2, 1/q^2
    T GMh, rs, irs;     // NFW halo
    T lcE0, lcEinv;     // uniform-E Lc table: first energy, 1 / spacing
};

// x unchanged, but opaque to the optimiser: conditions derived from a uniform
// value are then evaluated where they are used (a few scalar instructions)
// instead of being hoisted to the kernel entry and held in scalar registers
// across the whole particle loop.
template <typename X>
__device__ __forceinline__ X opaque(X x) {
    asm volatile("" : "+s"(x));
    return x;
}

// One binning of the observation layout.  Grids: sx, sy = n / width give the
// fast FP32 bin coordinate (the FP64 decision uses the defining form
// (v - x0) / width * n with the constants in Exact); shells and annuli: nb + 1
// edges from edge0 of the edge tables.  mom packs the listed moment codes in
// 3-bit fields: code m is (mom >> 3m) & 7 (0 mass, 1 v_los, 2 v_los^2, 3..6
// Gauss-Hermite h1..h4, whose bins' (V, 1/sigma) pairs start at pair gh0 of the
// Gauss-Hermite table).
constexpr int kMomBits = 3;
template <typename T>
struct BinDesc {
    int32_t kind, nmom, mom, off;   // off: first observable index of the binning
    int32_t nb, edge0, nx, ny;      // nb: bins per moment
    int32_t gh0, geo;   // geo: shells/annuli with log-spaced edges, ln e_k = x0 + k / sx
    T x0, sx, y0, sy;
    // FP32 grid guard terms (bins): gx0 = 2u sx |x0|, gy0 = 2u sy |y0| (the
    // rounded origins), gys = 6u sy (the rounded projection, per unit of
    // |y cos i| + |z sin i|)
    T gx0, gy0, gys;
};

template <typename T>
struct Layout {
    T cosi, sini;
    int32_t nbin;
    int32_t J;
    int32_t has_gh, ngh;   // Gauss-Hermite moments listed; pairs in the table
    BinDesc<T> b[kMaxBin];
};

// Compile-time signature of a layout's structure: nbin in the low 4 bits, then
// 13 bits per binning (kind 2, nmom 2, mom 9).  Kernels compiled for a signature
// take these from the signature instead of the layout (0: from the layout).
constexpr int kCodeBits = 13;
constexpr uint64_t bin_code(int kind, int nmom, int mom) { return uint64_t(kind | nmom << 2 | mom << 4); }
constexpr uint64_t layout_sig(int nbin, uint64_t c0, uint64_t c1 = 0, uint64_t c2 = 0, uint64_t c3 = 0) {
    return uint64_t(nbin) | c0 << 4 | c1 << (4 + kCodeBits) | c2 << (4 + 2 * kCodeBits) | c3 << (4 + 3 * kCodeBits);
}
constexpr int moms(int m0, int m1 = 0, int m2 = 0) { return m0 | m1 << kMomBits | m2 << (2 * kMomBits); }
// The layouts with compiled kernels: sky pixels (mass) with a kinematic grid
// (first and second LOS moments), alone or followed by 3D shells (mass); 3D
// shells (mass) with projected annuli (second LOS moment).
constexpr uint64_t kSigPixKin = layout_sig(2, bin_code(3, 1, moms(0)), bin_code(3, 2, moms(1, 2)));
constexpr uint64_t kSigPixKinShell =
    layout_sig(3, bin_code(3, 1, moms(0)), bin_code(3, 2, moms(1, 2)), bin_code(1, 1, moms(0)));
constexpr uint64_t kSigShellAnn = layout_sig(2, bin_code(1, 1, moms(0)), bin_code(2, 1, moms(2)));

// Structure of the layout seen by a kernel compiled for signature SIG.
template <uint64_t SIG, typename T>
struct LayoutView {
    const Layout<T>& L;
    __device__ __forceinline__ int nbin() const {
        if constexpr (SIG != 0) return int(SIG & 15);
        else return opaque(L.nbin);
    }
    __device__ __forceinline__ int kind(int b) const {
        if constexpr (SIG != 0) return int((SIG >> (4 + kCodeBits * b)) & 3);
        else return opaque(L.b[b].kind);
    }
    __device__ __forceinline__ int nmom(int b) const {
        if constexpr (SIG != 0) return int((SIG >> (6 + kCodeBits * b)) & 3);
        else return opaque(L.b[b].nmom);
    }
    __device__ __forceinline__ int mom(int b) const {
        if constexpr (SIG != 0) return int((SIG >> (8 + kCodeBits * b)) & 511);
        else return opaque(L.b[b].mom);
    }
    // does any binning list a Gauss-Hermite moment (code >= 3)?
    __device__ __forceinline__ bool has_gh() const {
        if constexpr (SIG != 0) return false;   // (the compiled signatures list none)
        else return opaque(L.has_gh) != 0;
    }
};

// Moving-prior cell geometry.
struct Cells {
    int32_t n0, n1, n2;   // cells along E, L/Lc or Lz/Lc, Lz/L
    int32_t ax2;          // 0: L/Lc in [0,1]; 1: Lz/Lc in [-1,1]
    int32_t ncell;
};

// FP64 tables and constants of the exact (re-)decision path, in device
// memory (read only when a decision is re-taken, or by the FP64 kernels).
struct Exact {
    Layout<float> lay;        // the layout as the FP32 kernels see it
    Cells cells;
    const Pot<double>* pots;
    const double* lctab;      // kLcTab per model
    const double* erange;     // Emin, Emax per model
    const double* edges;      // edge values
    const float* rce;         // kLcE values ln r_c(E_k) per model: Newton seeds (FP32 path)
    const float* gh;          // Gauss-Hermite table: (V, 1/sigma) per bin of each GH binning (FP32)
    double cosd, sind;
    double x0d[kMaxBin], wxd[kMaxBin], y0d[kMaxBin], wyd[kMaxBin];
};

// ------------------------------------------------------------------ potentials
template <typename T> __device__ __forceinline__ T dsqrt(T v) { return sqrt(v); }
template <typename T> __device__ __forceinline__ T dlog(T v) { return log(v); }
template <typename T> __device__ __forceinline__ T dexp(T v) { return exp(v); }
template <typename T> __device__ __forceinline__ T dlog1p(T v) { return log1p(v); }
// Fast forms for quantities that only feed guarded decisions or the orbit
// integration (a few ulp in FP32; exact IEEE forms in FP64).
// (a times the hardware reciprocal, 1 ulp: __fdividef still expands to the IEEE
// division sequence here)
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float qlog(float v) { return __logf(v); }
__device__ __forceinline__ double qlog(double v) { return log(v); }
__device__ __forceinline__ float qexp(float v) { return __expf(v); }
// ln of a weight ratio for the update (not a decision input): the hardware base-2
// logarithm times ln 2 (the ratio is a normal number)
__device__ __forceinline__ float qlog_ratio(float v) { return __builtin_amdgcn_logf(v) * 0.693147180559945309f; }
__device__ __forceinline__ double qlog_ratio(double v) { return log(v); }
__device__ __forceinline__ double qexp(double v) { return exp(v); }
// Square root and ln(1 + x) of the FP32 potentials: the hardware square root
// (at most 1.6u relative error, u = 2^-24, measured on gfx950 over every float in
// [2^-30, 2^30)), and ln(1 + x) = x ln(w) / (w - 1) with w = 1 + x rounded
// (Goldberg 1991, "What every computer scientist should know about
// floating-point arithmetic", Theorem 4), ln(w) from the hardware base-2
// logarithm (at most 6u relative error over the same floats).  The FP64 kernels
// use the library forms.
__device__ __forceinline__ float psqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double psqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float plog1p(float v) {
    const float w = 1.0f + v;
    const float d = w - 1.0f;
    const float l = __builtin_amdgcn_logf(w) * 0.693147180559945309f;
    return d == 0.0f ? v : v * (l * __builtin_amdgcn_rcpf(d));
}
__device__ __forceinline__ double plog1p(double v) { return log1p(v); }

// Phi(x) and a = -grad Phi.  POT is the compile-time potential kind.
template <int POT, typename T>
__device__ __forceinline__ void potential(const Pot<T>& p, T x, T y, T z, T& phi, T& ax, T& ay, T& az) {
    if (POT == 1) {   // logarithmic
        const T s = p.Rc2 + x * x + y * y + z * z * p.iq2;
        const T f = qdiv(p.v2, s);
        phi = T(0.5) * p.v2 * qlog(s);
        ax = -f * x;
        ay = -f * y;
        az = -f * z * p.iq2;
        return;
    }
    const T r2 = x * x + y * y + z * z;
    const T r = psqrt(r2);
    const T u = r + p.a;
    T ph = -qdiv(p.GM, u);
    T g_over_r = r > T(0) ? qdiv(p.GM, u * u * r) : T(0);   // (dPhi/dr)/r
    if (POT == 2 && p.GMh > T(0)) {
        const T xx = r * p.irs;
        const T l1 = plog1p(xx);
        // dPhi_NFW/dr = G Mh/rs^2 f(x), f = ln(1+x)/x^2 - 1/(x(1+x)); the two terms
        // cancel near x = 0, where the Taylor series is used instead.
        T f;
        if constexpr (sizeof(T) == 4) {
            // one hardware reciprocal of r serves every division (1/x = rs/r)
            const T ir = r > T(0) ? qdiv(T(1), r) : T(0);
            ph += r > T(0) ? -p.GMh * l1 * ir : -p.GMh * p.irs;
            if (xx < T(0.05)) {
                f = T(0.5) + xx * (T(-2.0 / 3.0) + xx * (T(0.75) + xx * (T(-0.8) + xx * (T(5.0 / 6.0) - xx * T(6.0 / 7.0)))));
            } else {
                const T ix = p.rs * ir;
                f = ix * (l1 * ix - qdiv(T(1), T(1) + xx));
            }
            g_over_r += p.GMh * p.irs * p.irs * f * ir;
        } else {
            ph += r > T(0) ? -p.GMh * l1 / r : -p.GMh * p.irs;
            if (xx < T(0.05)) {
                f = T(0.5) + xx * (T(-2.0 / 3.0) + xx * (T(0.75) + xx * (T(-0.8) + xx * (T(5.0 / 6.0) - xx * T(6.0 / 7.0)))));
            } else {
                f = l1 / (xx * xx) - T(1) / (xx * (T(1) + xx));
            }
            g_over_r += r > T(0) ? p.GMh * p.irs * p.irs * f / r : T(0);
        }
    }
    phi = ph;
    ax = -g_over_r * x;
    ay = -g_over_r * y;
    az = -g_over_r * z;
}

// Equatorial Phi(R), dPhi/dR and d2Phi/dR2 (circular-orbit Newton iteration).
template <int POT, typename T>
__device__ __forceinline__ void radial_derivs(const Pot<T>& p, T r, T& phi, T& d1, T& d2) {
    if (POT == 1) {
        const T s = p.Rc2 + r * r;
        phi = T(0.5) * p.v2 * dlog(s);
        d1 = p.v2 * r / s;
        d2 = p.v2 * (p.Rc2 - r * r) / (s * s);
        return;
    }
    const T u = r + p.a;
    phi = -p.GM / u;
    d1 = p.GM / (u * u);
    d2 = T(-2) * p.GM / (u * u * u);
    if (POT == 2 && p.GMh > T(0)) {
        const T l1 = dlog1p(r * p.irs);
        const T rrs = r + p.rs;
        phi += -p.GMh * l1 / r;
        d1 += p.GMh * (l1 / (r * r) - T(1) / (r * rrs));
        d2 += p.GMh * (T(1) / (r * r * rrs) + (T(2) * r + p.rs) / (r * r * rrs * rrs) - T(2) * l1 / (r * r * r));
    }
}

// Angular momentum Lc(E) of the circular orbit of energy E.  Radii are
// bracketed to [1e-8, 1e8]; energies outside take the end values.
//   Hernquist: 2E u^2 + GM u + GM a = 0 with u = r_c + a, in the stable form
//     r_c = 4a(GM + E a)/(sqrt(GM^2 - 8 E GM a) - GM - 4 E a);
//   otherwise: E_c(r_k) tabulated at kLcTab log-spaced radii, r from the table by
//     bisection and linear interpolation in ln r, then Newton steps on
//     E_c(r) = Phi + r Phi'/2 = E with dE_c/dr = (3 Phi' + r Phi'')/2.
template <int POT, typename T, int NEWTON>
__device__ __forceinline__ T circular_L(const Pot<T>& p, const T* __restrict__ tab, T E) {
    if (POT == 0) {
        if (!(E < T(0))) return T(-1);        // unbound: infinite Lc
        const T D = p.GM * p.GM - T(8) * E * p.GM * p.a;
        const T rc = T(4) * p.a * (p.GM + E * p.a) / (dsqrt(D) - p.GM - T(4) * E * p.a);
        if (!(rc > T(0))) return T(0);
        return rc * dsqrt(p.GM * rc) / (rc + p.a);
    } else {
        const T lr0 = T(-8.0 * 2.302585092994046), dl = T(16.0 * 2.302585092994046 / (kLcTab - 1));
        T r;
        if (E <= tab[0]) {
            r = T(1e-8);
        } else if (E >= tab[kLcTab - 1]) {
            r = T(1e8);
        } else {
            int lo = 0, hi = kLcTab - 1;
            #pragma unroll
            for (int it = 0; it < 8; ++it) {
                const int mid = (lo + hi) >> 1;
                if (tab[mid] <= E) lo = mid; else hi = mid;
            }
            const T t = (E - tab[lo]) / (tab[hi] - tab[lo]);
            r = dexp(lr0 + (T(lo) + t) * dl);
            #pragma unroll
            for (int it = 0; it < NEWTON; ++it) {
                T ph, d1, d2;
                radial_derivs<POT, T>(p, r, ph, d1, d2);
                const T Ec = ph + T(0.5) * r * d1;
                const T dE = T(0.5) * (T(3) * d1 + r * d2);
                r = r - (Ec - E) / dE;
            }
        }
        T ph, d1, d2;
        radial_derivs<POT, T>(p, r, ph, d1, d2);
        return r * dsqrt(r * d1);
    }
}

__device__ __forceinline__ int clamp_cell(double f, int n) {
    if (!(f >= 0.0)) return 0;   // also NaN
    if (f >= double(n)) return n - 1;
    return int(f);
}
__device__ __forceinline__ int clamp_cell(float f, int n) {
    // (branch free: max(NaN, 0) is 0, and the conversion saturates large values)
    return min(int(fmaxf(f, 0.0f)), n - 1);
}
// Is the clamped FP32 coordinate f within g of a cell edge it could cross?
// (Branch free: every term is evaluated and combined with selects, so that the
// test costs a few VALU operations and no exec-mask branches.)
__device__ __forceinline__ bool near_cell_edge(float f, int n, float g) {
    const float fr = f - floorf(f);
    const bool inside = (f > -g) & (f < float(n) + g);   // (false for NaN)
    const bool edge = (fr < g) | (fr > 1.0f - g);
    return inside ? edge : (f != f);                      // far outside: clamped either way
}

// Cell index from E, L, Lz and Lc(E) in FP64 (the defining arithmetic): E
// uniform over [Emin, Emax], then L/Lc in [0, 1] or Lz/Lc in [-1, 1], then
// optionally Lz/L in [-1, 1]; coordinates outside a range take the edge cell.
// Lc < 0 marks an unbound energy (infinite Lc), Lc = 0 a degenerate one.
__device__ __forceinline__ int cell_axis_E(const Cells& c, double Emin, double Emax, double E) {
    return clamp_cell((E - Emin) / (Emax - Emin) * c.n0, c.n0);
}
__device__ __forceinline__ int cell_axis_2(const Cells& c, double L, double Lz, double Lc) {
    if (c.ax2 == 0) return clamp_cell((Lc > 0 ? L / Lc : (Lc < 0 ? 0.0 : 1e300)) * c.n1, c.n1);
    return clamp_cell(((Lc > 0 ? Lz / Lc : (Lc < 0 ? 0.0 : (Lz > 0 ? 1e300 : -1e300))) + 1.0) * 0.5 * c.n1, c.n1);
}
__device__ __forceinline__ int cell_axis_3(const Cells& c, double L, double Lz) {
    return c.n2 > 1 ? clamp_cell(((L > 0 ? Lz / L : 0.0) + 1.0) * 0.5 * c.n2, c.n2) : 0;
}
__device__ __forceinline__ int cell_index(const Cells& c, double Emin, double Emax, double E, double L, double Lz,
                                          double Lc) {
    return (cell_axis_E(c, Emin, Emax, E) * c.n1 + cell_axis_2(c, L, Lz, Lc)) * c.n2 + cell_axis_3(c, L, Lz);
}

// Cell of the moving prior in FP64, Lc(E) from the circular-orbit table.
template <int POT>
__device__ __forceinline__ int prior_cell_f64(const Pot<double>& p, const double* __restrict__ tab, const Cells& c,
                                              double Emin, double Emax, double x, double y, double z, double vx,
                                              double vy, double vz) {
    double phi, ax, ay, az;
    potential<POT, double>(p, x, y, z, phi, ax, ay, az);
    const double E = 0.5 * (vx * vx + vy * vy + vz * vz) + phi;
    const double Lx = y * vz - z * vy, Ly = z * vx - x * vz, Lz = x * vy - y * vx;
    const double L = sqrt(Lx * Lx + Ly * Ly + Lz * Lz);
    return cell_index(c, Emin, Emax, E, L, Lz, circular_L<POT, double, 5>(p, tab, E));
}

// E, |L|, Lz and Lc(E) in FP64, the integrals of motion the priors are computed
// over.  Lc(E) from Newton steps on E_c(r) = E seeded by the tabulated ln r_c(E)
// (uniform in E from E0 with 1/spacing invh; the seed is good to about 1e-6, so
// three steps reach FP64 precision), the Hernquist closed form, or the
// circular-orbit table (gtab, device memory) outside the seed table.
template <int POT>
__device__ __forceinline__ double energy64(const Pot<double>& p, double x, double y, double z, double vx, double vy,
                                          double vz) {
    double phi, ax, ay, az;
    potential<POT, double>(p, x, y, z, phi, ax, ay, az);
    return 0.5 * (vx * vx + vy * vy + vz * vz) + phi;
}
__device__ __forceinline__ void angmom64(double x, double y, double z, double vx, double vy, double vz, double& L,
                                         double& Lz) {
    const double Lx = y * vz - z * vy, Ly = z * vx - x * vz;
    Lz = x * vy - y * vx;
    L = sqrt(Lx * Lx + Ly * Ly + Lz * Lz);
}
template <int POT>
__device__ __forceinline__ double lc_seeded(const Pot<double>& p, const double* __restrict__ gtab,
                                           const float* __restrict__ rce, double E0, double invh, double E) {
    const double t = (E - E0) * invh;
    if (POT == 0 || !(t >= 0.0) || !(t < double(kLcE - 1))) return circular_L<POT, double, 5>(p, gtab, E);
    const int k = int(t);
    double r = exp(double(rce[k]) + (t - k) * double(rce[k + 1] - rce[k]));
    #pragma unroll
    for (int it = 0; it < 3; ++it) {
        double ph, d1, d2;
        radial_derivs<POT, double>(p, r, ph, d1, d2);
        r = r - (ph + 0.5 * r * d1 - E) / (0.5 * (3.0 * d1 + r * d2));
    }
    double ph, d1, d2;
    radial_derivs<POT, double>(p, r, ph, d1, d2);
    return r * sqrt(r * d1);
}
template <int POT>
__device__ __forceinline__ void integrals_seeded(const Pot<double>& p, const double* __restrict__ gtab,
                                                 const float* __restrict__ rce, double E0, double invh, double x,
                                                 double y, double z, double vx, double vy, double vz, double& E,
                                                 double& L, double& Lz, double& Lc) {
    E = energy64<POT>(p, x, y, z, vx, vy, vz);
    angmom64(x, y, z, vx, vy, vz, L, Lz);
    Lc = lc_seeded<POT>(p, gtab, rce, E0, invh, E);
}

// Cell of the moving prior in FP64 for a decision the FP32 path left open.
template <int POT>
__device__ __forceinline__ int prior_cell_seeded(const Pot<double>& p, const double* __restrict__ gtab,
                                              const float* __restrict__ rce, double E0, double invh, const Cells& c,
                                              double Emin, double Emax, double x, double y, double z, double vx,
                                              double vy, double vz) {
    double E, L, Lz, Lc;
    integrals_seeded<POT>(p, gtab, rce, E0, invh, x, y, z, vx, vy, vz, E, L, Lz, Lc);
    return cell_index(c, Emin, Emax, E, L, Lz, Lc);
}

// Lc(E) of an FP32 kernel from the model's uniform-E table: pairs (ln Lc(E_k),
// bound) at E_k = E0 + k / invh, k < kLcE; ln Lc is interpolated linearly and
// bound is the relative interpolation error on [E_k, E_k+1] (measured on the
// host in FP64, with a safety factor).  dl receives a bound on the relative
// error of the FP32 result: the interpolation bound; the energy error eE, the
// rounding of E0 and of the table index (3u |E - E0|) through the slope of
// ln Lc; the rounding of the interpolated logarithm and of the hardware exp.
// Returns false outside the table.
__device__ __forceinline__ bool lc_from_table(const float2* __restrict__ et, float E0, float invh, float E, float eE,
                                              float& Lc, float& dl) {
    const float d = E - E0;
    const float t = d * invh;
    if (!(t >= 0.0f) || !(t < float(kLcE - 1))) return false;
    const int k = int(t);
    const float f = t - float(k);
    const float2 a = et[k], b = et[k + 1];
    const float l = a.x + f * (b.x - a.x);
    Lc = __expf(l);
    dl = a.y + fabsf(b.x - a.x) * invh * (eE + kU32 * (fabsf(E0) + 3.0f * fabsf(d))) +
         kU32 * (4.0f * fabsf(l) + 3.0f);
    return true;
}

// Guard of the energy axis of the prior cells, per model: the FP32 coordinate
// fE = (E - Emin) sE differs from the exact one by at most
//   sE (eE + u |Emin|) + |fE| (4u + u (|Emin| + |Emax|) / (Emax - Emin))
// (eE: the energy error; the rounded Emin; the difference, the product and
// the rounded sE, itself n0 over the difference of the rounded range); the
// guard is twice that, plus a floor.
struct CellGuard {
    float e0, e1, e2;   // gE = e0 + e1 eE + e2 |fE|
};
__device__ __forceinline__ CellGuard cell_guard(float Emin, float Emax, float sE) {
    CellGuard g;
    g.e0 = 2.0f * sE * kU32 * fabsf(Emin) + kGuardBinFloor;
    g.e1 = 2.0f * sE;
    g.e2 = 2.0f * kU32 * (4.0f + (fabsf(Emin) + fabsf(Emax)) / (Emax - Emin));
    return g;
}

// Cell of the moving prior from FP32 values: kinetic energy KE and potential
// phi (E = KE + phi), position and velocity.  Returns the axes whose FP32
// coordinate lies within the guard band of a cell edge (bit 0: E, bit 1: L/Lc
// or Lz/Lc, also when Lc(E) is not in the table or not positive, bit 2: Lz/L);
// the caller re-decides those in FP64.  cell is the index from the clamped FP32
// coordinates of every axis (exact on the axes not returned).
// Guards, twice a bound on the FP32 error (u = 2^-24):
//   E: |E32 - E| <= u (4 KE + 25 |phi| + 3 v0^2): the kinetic sum, the
//      potential (at most 24u |phi| for the analytic potentials with the
//      hardware reciprocal, logarithm and square root: the Hernquist+NFW sum is
//      the largest, r 3.1u, x = r/rs 5.1u, ln(1+x) 11.1u, 1/r 4.6u, the NFW
//      term 18.7u, the Hernquist term 8.6u, the sum 19.7u; plus 3u v0^2 from
//      the argument of the logarithmic potential's log) and the sum; see
//      cell_guard;
//   L/Lc or Lz/Lc: the rounding of L (2u per product pair; the sum of squares
//      and the hardware root 4u L) or Lz
//      (2u (|x vy| + |y vx|)) over Lc, and the relative error of Lc (dl, plus
//      3u for the reciprocal and the product) times the coordinate's distance
//      from the axis origin, plus 2u |f2|;
//   Lz/L: 1e-4 cells.
// Cell-axis configurations a kernel can be compiled for (CAX): the second axis
// and the presence of the third taken from the Cells at run time (0), or fixed:
// Lz/Lc with no third axis (1), L/Lc with no third axis (2).
constexpr int kCaxRuntime = 0, kCaxLzNo3 = 1, kCaxLNo3 = 2;

// The compiled configuration matching a prior's cells (kCaxRuntime if none).
__host__ __device__ inline int cax_of(const Cells& c) {
    if (c.n2 == 1 && c.ax2 == 1) return kCaxLzNo3;
    if (c.n2 == 1 && c.ax2 == 0) return kCaxLNo3;
    return kCaxRuntime;
}

template <int POT, int CAX = kCaxRuntime>
__device__ __forceinline__ unsigned cell_fast(const Pot<float>& p, const float2* __restrict__ et, const Cells& c,
                                              float Emin, float sE, const CellGuard& G, float KE, float phi, float x,
                                              float y, float z, float vx, float vy, float vz, int& cell) {
    const int n0 = opaque(c.n0), n1 = opaque(c.n1);
    const int n2 = CAX == kCaxRuntime ? opaque(c.n2) : 1;
    const int ax2 = CAX == kCaxRuntime ? opaque(c.ax2) : (CAX == kCaxLzNo3 ? 1 : 0);
    const float E = KE + phi;
    const float eE = kU32 * (4.0f * KE + 25.0f * fabsf(phi) + 3.0f * p.v2);
    const float xvy = x * vy, yvx = y * vx;
    const float Lz = xvy - yvx;
    float L = 0.0f, dL = 2.0f * kU32 * (fabsf(xvy) + fabsf(yvx));
    if (ax2 == 0 || n2 > 1) {   // |L| only for the L/Lc and Lz/L axes
        const float yvz = y * vz, zvy = z * vy, zvx = z * vx, xvz = x * vz;
        const float Lx = yvz - zvy, Ly = zvx - xvz;
        L = __builtin_amdgcn_sqrtf(Lx * Lx + Ly * Ly + Lz * Lz);
        if (ax2 == 0) dL += 2.0f * kU32 * (fabsf(yvz) + fabsf(zvy) + fabsf(zvx) + fabsf(xvz)) + 4.0f * kU32 * L;
    }
    float Lc = 1.0f, dl = 1.0f;
    const bool have = lc_from_table(et, p.lcE0, p.lcEinv, E, eE, Lc, dl) && Lc > 0.0f;
    const float fE = (E - Emin) * sE;
    const float iLc = qdiv(1.0f, Lc);
    const float s2 = ax2 == 0 ? float(n1) : 0.5f * float(n1);
    const float f2 = ax2 == 0 ? L * iLc * float(n1) : (Lz * iLc + 1.0f) * s2;
    const float f3 = n2 > 1 ? ((L > 0.0f ? qdiv(Lz, L) : 0.0f) + 1.0f) * 0.5f * float(n2) : 0.5f;
    const float gE = G.e0 + G.e1 * eE + G.e2 * fabsf(fE);
    const float g2 = 2.0f * (s2 * dL * iLc + fabsf(f2 - (ax2 == 0 ? 0.0f : s2)) * (dl + 3.0f * kU32) +
                             2.0f * kU32 * fabsf(f2)) + kGuardBinFloor;
    unsigned open = near_cell_edge(fE, n0, gE) ? 1u : 0u;
    open |= (!have || near_cell_edge(f2, n1, g2)) ? 2u : 0u;
    open |= (n2 > 1 && near_cell_edge(f3, n2, kGuardCell)) ? 4u : 0u;
    cell = (clamp_cell(fE, n0) * n1 + (have ? clamp_cell(f2, n1) : 0)) * n2 + (n2 > 1 ? clamp_cell(f3, n2) : 0);
    return open;
}

// ---------------------------------------------------------------- observables
// Bin of value v against ne increasing edges: -1 outside [e0, e_last).
template <typename T>
__device__ __forceinline__ int edge_bin(const T* __restrict__ e, int ne, T v) {
    if (!(v >= e[0]) || !(v < e[ne - 1])) return -1;
    int lo = 0, hi = ne - 1;   // e[lo] <= v < e[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (v >= e[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

// Bin of one binning in FP64, the defining arithmetic: grid pixel
// floor((v - x0) / width * n) on the sky plane, or the edge interval of r / R.
__device__ __forceinline__ int bin_f64(int kind, double cosd, double sind, double x0, double wx, int nx, double y0,
                                       double wy, int ny, const double* __restrict__ e, int ne, double x, double y,
                                       double z) {
    const double X = x, Ys = y * cosd - z * sind;
    if (kind == 3) {
        const double fx = floor((X - x0) / wx * nx);
        const double fy = floor((Ys - y0) / wy * ny);
        if (fx >= 0 && fx < nx && fy >= 0 && fy < ny) return int(fy) * nx + int(fx);
        return -1;
    }
    const double rad = kind == 1 ? sqrt(x * x + y * y + z * z) : sqrt(X * X + Ys * Ys);
    return edge_bin(e, ne, rad);
}

// Bin of binning b (kind `kind`) in FP32, -1 outside; sure = false when the
// coordinate lies within the guard band of an edge (the caller re-decides with
// bin_f64).  Ys = y cos i - z sin i in FP32 and aYs = |y cos i| + |z sin i|.
// Guards (twice the bound, u = 2^-24):
//   grid x: fx = (x - x0) sx carries the rounding of x0 (u |x0| sx) and three
//     relative roundings (the difference, sx, the product): 2(u sx |x0| + 3u |fx|);
//   grid y: the same plus the projection, two roundings per product (cos i or
//     sin i, the product) and one of the difference, <= 3u aYs, times sy;
//   radius: the sum of squares (3u, halved by the root), the hardware root
//     (at most 1.6u, counted as 2u) and the rounded edge (u) stay below 12u r;
//     the projected radius adds 6u aYs.
__device__ __forceinline__ int bin_fast(const BinDesc<float>& d, int kind, const float* __restrict__ ef, float x,
                                        float y, float z, float Ys, float aYs, bool& sure) {
    if (kind == 3) {
        const float fx = (x - d.x0) * d.sx;
        const float fy = (Ys - d.y0) * d.sy;
        const float gx = d.gx0 + 6.0f * kU32 * fabsf(fx) + kGuardBinFloor;
        const float gy = d.gy0 + d.gys * aYs + 6.0f * kU32 * fabsf(fy) + kGuardBinFloor;
        sure = !(near_cell_edge(fx, d.nx, gx) | near_cell_edge(fy, d.ny, gy));
        const bool in = (fx >= 0.0f) & (fx < float(d.nx)) & (fy >= 0.0f) & (fy < float(d.ny));
        // (the conversions of out-of-range values are not used)
        return in ? int(fy) * d.nx + int(fx) : -1;
    }
    const float rad = kind == 1 ? psqrt(x * x + y * y + z * z) : psqrt(x * x + Ys * Ys);
    const float* e = ef + d.edge0;
    const int ne = d.nb + 1;
    const float g = 12.0f * kU32 * rad + (kind == 1 ? 0.0f : 6.0f * kU32 * aYs);
    int k;
    if (d.geo) {
        // log-spaced edges: the bin from ln r (within one bin of the right one, as
        // the host checked), then one step down and one up by comparing with the
        // edges themselves, so that k is the edge interval a search would find
        const bool in = (rad >= e[0]) & (rad < e[ne - 1]);
        int j = int(fminf(fmaxf((qlog(rad) - d.x0) * d.sx, 0.0f), float(d.nb - 1)));
        j -= int(rad < e[j]);
        j += int(rad >= e[j + 1]);
        k = in ? j : -1;
    } else {
        k = edge_bin(e, ne, rad);
    }
    if (k >= 0) sure = !(rad - e[k] < g) && !(e[k + 1] - rad < g);
    else sure = !(fabsf(rad - e[0]) < g) && !(fabsf(rad - e[ne - 1]) < g) && rad == rad;
    return k;
}

// Line-of-sight velocity v_los = vy sin i + vz cos i (one fused form everywhere,
// so that every path of a kernel computes the same value).
__device__ __forceinline__ float line_of_sight(float vy, float vz, float sini, float cosi) {
    return fmaf(vy, sini, vz * cosi);
}
__device__ __forceinline__ double line_of_sight(double vy, double vz, double sini, double cosi) {
    return vy * sini + vz * cosi;
}

// Kernel value of moment code mo (0: 1, 1: v_los, 2: v_los^2).
template <typename T>
__device__ __forceinline__ T moment_value(int mo, T vl) {
    return mo == 0 ? T(1) : (mo == 1 ? vl : vl * vl);
}

// Gauss-Hermite kernel (section 1: absorption-line kinematics; the LOSVD of a
// bin expanded about its Gaussian (V, sigma) as in van der Marel & Franx 1993):
// 2 sqrt(pi) alpha(nu) H_m(nu) = sqrt(2) exp(-nu^2/2) H_m(nu), nu = (v - V)/sigma,
// for m = code - 2 = 1..4, with the normalised Hermite polynomials written out:
//   m = 1: 2 nu,  m = 2: 2 nu^2 - 1,  m = 3: sqrt(2/3) (2 nu^3 - 3 nu),
//   m = 4: (4 nu^4 - 12 nu^2 + 3) / sqrt(12)   (each times exp(-nu^2/2)).
// gv: the bin's (V, 1/sigma).
template <typename T>
__device__ __forceinline__ T gh_value(int code, T vl, T V, T isig) {
    const T nu = (vl - V) * isig, n2 = nu * nu;
    const T e = qexp(T(-0.5) * n2);
    T p;
    if (code == 3) p = T(2) * nu;
    else if (code == 4) p = T(2) * n2 - T(1);
    else if (code == 5) p = T(0.816496580927726033) * nu * (T(2) * n2 - T(3));
    else p = T(0.288675134594812882) * (n2 * (T(4) * n2 - T(12)) + T(3));
    return p * e;
}

// Kernel value of any moment code; (V, 1/sigma) of the bin from gv (read only
// for the Gauss-Hermite codes).
template <typename T>
__device__ __forceinline__ T kernel_value(int code, T vl, const T* gv) {
    if (code <= 2) return moment_value<T>(code, vl);
    return gh_value<T>(code, vl, gv[0], gv[1]);
}

}  // namespace m2m
