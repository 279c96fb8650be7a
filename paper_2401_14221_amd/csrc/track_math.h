// Device arithmetic of one track-layer step, one lane per track, in FP32
// (the fit) or FP64 (the FP64 fit, every function templated on the type).
//
// State p = (x, y, z, ipt = 1/pT, phi, theta), charge q; covariance kept
// packed as 21 registers (lower triangle, row-major).  The step follows the
// method's order (paper, Section 2): propagate the state to the surface,
// transport the covariance with the Jacobian, then Kalman-update with the
// surface's 3D hit.  Formulas are the textbook helix in a uniform field and
// the linear Kalman filter; see the function comments for each form used.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p2r {

constexpr float KAPPA = 2.99792458e-3f;   // GeV / (T cm)
constexpr float PI_F = 3.14159265358979f;
constexpr float TWO_PI_F = 6.28318530717959f;
constexpr float INV_TWO_PI_F = 0.159154943091895f;
constexpr float HALF_PI_F = 1.57079632679490f;

enum : uint32_t {
    ST_NO_CROSSING = 1u << 0,
    ST_NEWTON_FAIL = 1u << 1,
    ST_FP64_FALLBACK = 1u << 2,
    ST_S_NOT_PD = 1u << 3,
    ST_BAD_INPUT = 1u << 4,
    ST_ML_REJECTED = 1u << 5,
    ST_HIT_MISSING = 1u << 6,
    ST_CHI2_CUT = 1u << 7,
    ST_DONE = 1u << 31,
};
constexpr int NUSED_SHIFT = 8;
// status bits 8..15: the number of applied updates, saturating at 255
__host__ __device__ __forceinline__ uint32_t nused_field(int nused) {
    return (uint32_t)(nused > 255 ? 255 : nused) << NUSED_SHIFT;
}

// Relative pivot thresholds of the positive-definiteness test of S (a
// pivot d_k must exceed tau * S_kk).  FP32: below 1e-3 the FP32 inverse
// would carry more than ~1e-4 relative error, so the FP64 inversion takes
// over.  FP64: S is formed from FP32 covariance values (relative error
// >= 6e-8), so pivots below 1e-6 of the diagonal carry no information and S
// is treated as singular.
constexpr float PD_TAU32 = 1e-3f;
constexpr double PD_TAU64 = 1e-6;
// The FP64 fit (every step in FP64) takes the oracle's threshold.
constexpr double PD_TAU_F64_FIT = 1e-12;

// Reciprocal and quotient: v_rcp_f32 (1 ulp) followed by one Newton
// correction of the result, r + r (1 - b r) and q + r (a - b q) with the
// residuals formed exactly by FMA.  The result is within 1 ulp and almost
// always the correctly rounded one, in 3-4 instructions instead of the ~17
// of the IEEE sequence, whose extra steps only rescale operands near the
// denormal and overflow ranges (the fit's operands are lengths, angles and
// their ratios, far from both).  A bare v_rcp_f32 is not enough: its extra
// rounding moves propagated positions by a few ulp, a visible fraction of
// a 100 um hit's residual at r ~ 100 cm.
__device__ __forceinline__ float frcp(float b) {
    const float r = __builtin_amdgcn_rcpf(b);
    return fmaf(fmaf(-b, r, 1.0f), r, r);
}
__device__ __forceinline__ float fdiv(float a, float b) {
    const float r = __builtin_amdgcn_rcpf(b);
    const float q = a * r;
    return fmaf(fmaf(-b, q, a), r, q);
}

// Square root for starting values only (v_sqrt_f32, 1 ulp): the iteration
// that follows removes its error.
__device__ __forceinline__ float sqrt_start(float x) { return __builtin_amdgcn_sqrtf(x); }

// sin and cos of x for |x| <= 1e4 (larger arguments take the library
// routine): x = k pi/2 + r with pi/2 split in three FP32 parts (Cody and
// Waite's reduction, each product subtracted by FMA), |r| <= pi/4, then the
// Taylor series of sin r to r^9 and cos r to r^10 (truncation below 3e-9)
// and the quadrant's swap and signs.  Within 1.5 ulp of the exact values.
__device__ __forceinline__ void sincos_fit(float x, float* sn, float* cs) {
    if (!(fabsf(x) <= 1.0e4f)) { sincosf(x, sn, cs); return; }
    const float k = rintf(x * 0.636619746685028f);                 // 2/pi
    float r = fmaf(k, -1.5707963705062866f, x);                     // pi/2 = C1 + C2 + C3
    r = fmaf(k, 4.371138828673793e-08f, r);
    r = fmaf(k, 1.7763568394002505e-15f, r);
    const float r2 = r * r;
    float ps = fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f);
    ps = fmaf(r2, ps, 1.0f / 120.0f);
    ps = fmaf(r2, ps, -1.0f / 6.0f);
    const float sr = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    pc = fmaf(r2, pc, -1.0f / 720.0f);
    pc = fmaf(r2, pc, 1.0f / 24.0f);
    pc = fmaf(r2, pc, -0.5f);
    const float cr = fmaf(r2, pc, 1.0f);
    const int q = (int)k;
    const float a = (q & 1) ? cr : sr;      // sin: sr, cr, -sr, -cr for q = 0..3
    const float b = (q & 1) ? sr : cr;      // cos: cr, -sr, -cr, sr
    *sn = (q & 2) ? -a : a;
    *cs = ((q + 1) & 2) ? -b : b;
}

// Numeric helpers of the templated arithmetic below: FP32 uses the short
// forms above, FP64 the library's correctly rounded ones.
__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float div_(float a, float b) { return fdiv(a, b); }
__device__ __forceinline__ double div_(double a, double b) { return a / b; }
__device__ __forceinline__ float rcp_(float b) { return frcp(b); }
__device__ __forceinline__ double rcp_(double b) { return 1.0 / b; }
__device__ __forceinline__ float sqrt_start_(float x) { return sqrt_start(x); }
__device__ __forceinline__ double sqrt_start_(double x) { return sqrt(x); }
__device__ __forceinline__ void sincos_(float x, float* s, float* c) { sincos_fit(x, s, c); }
__device__ __forceinline__ void sincos_(double x, double* s, double* c) { sincos(x, s, c); }
template <typename T> __device__ __forceinline__ constexpr T pi_() { return T(3.14159265358979323846); }
template <typename T> __device__ __forceinline__ constexpr T two_pi_() { return T(6.28318530717958647692); }

// packed index of (i, j), j <= i
constexpr int I21(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

struct Params {
    float bz;
    float tol;
    int32_t max_iter;
    float chi2_cut;
    int32_t fp64_fallback;
    int32_t start_mode;   // cylinder start: 0 straight line (plain), 1 closed form
};

// lo: the low parts of the compensated components of an FP32 state (below).
template <typename T>
struct StateT {
    T p[6];
    T c[21];
    T q;
    T lo[6] = {};
};
using State = StateT<float>;

// ------------------------------------------------------ compensated state
// An FP32 fit that rounds its state to FP32 after every propagation and
// update loses, at r ~ 100 cm, 0.04 um of position per rounding, and for
// theta near pi (ulp 2.4e-7 rad) the crossing of the next plane moves by
// (Z - z) dtheta / cos^2(theta): over 20 layers enough to move the chi2 sum
// of 100 um hits by 1e-3 of itself.  So the positions and angles (x, y, z,
// phi, theta) are carried as unevaluated sums p[i] + lo[i] of two floats:
// every increment is added with Dekker's Fast2Sum, whose rounding error goes
// to lo[i]; residuals subtract lo[i]; the sines and cosines of phi and theta
// are corrected to first order in lo[i]; and each step ends by renormalising
// so that p[i] is the float nearest to the sum.  Fast2Sum is exact when
// |p[i]| >= |increment|; otherwise (a position near 0 moved by a larger step)
// it can lose up to half an ulp of the increment, no more than plain
// rounding would, at a point where that ulp is small.  1/pT and the
// covariance stay plain FP32.  The FP64 fit carries no low parts.
constexpr int N_COMP = 5;
__device__ __forceinline__ constexpr int comp_index(int k) { return k < 3 ? k : k + 1; }   // x y z phi theta

template <typename T>
__device__ __forceinline__ void add_to(StateT<T>& st, int i, T d) {
    if constexpr (sizeof(T) == sizeof(float)) {
        const T a = st.p[i];
        const T s = a + d;
        st.lo[i] += d - (s - a);
        st.p[i] = s;
    } else {
        st.p[i] += d;
    }
}

// p[i] <- the float nearest to p[i] + lo[i], lo[i] <- the remainder (z is
// left as it is: it enters only residuals and path lengths, which use the
// sum, and a plane resets it)
template <typename T>
__device__ __forceinline__ void renormalise(StateT<T>& st) {
    if constexpr (sizeof(T) == sizeof(float)) {
        constexpr int idx[4] = {0, 1, 4, 5};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = idx[k];
            const T s = st.p[i] + st.lo[i];
            st.lo[i] = st.lo[i] - (s - st.p[i]);
            st.p[i] = s;
        }
    }
}

// the parameters as FP32 values: each the float nearest to p[i] + lo[i]
template <typename T>
__device__ __forceinline__ void finalise(StateT<T>& st) {
    if constexpr (sizeof(T) == sizeof(float)) {
#pragma unroll
        for (int k = 0; k < N_COMP; ++k) {
            const int i = comp_index(k);
            st.p[i] += st.lo[i];
            st.lo[i] = T(0);
        }
    }
}

// m - (p[i] + lo[i])
template <typename T>
__device__ __forceinline__ T residual_of(const StateT<T>& st, int i, T m) {
    if constexpr (sizeof(T) == sizeof(float)) return (m - st.p[i]) - st.lo[i];
    else return m - st.p[i];
}

// sin and cos of p[i] + lo[i] from those of p[i], to first order in lo[i]
template <typename T>
__device__ __forceinline__ void sincos_comp(const StateT<T>& st, int i, T* sn, T* cs) {
    sincos_(st.p[i], sn, cs);
    if constexpr (sizeof(T) == sizeof(float)) {
        const T s0 = *sn, c0 = *cs, d = st.lo[i];
        *sn = fma_(c0, d, s0);
        *cs = fma_(-s0, d, c0);
    }
}

// ---------------------------------------------------------------- helix
// Point of the helix at transverse path s, in the half-angle form
//   u = omega s / 2,  chord = s sin(u)/u,  phi_m = phi + u,
//   x' = x + chord cos(phi_m),  y' = y + chord sin(phi_m),  phi' = phi + 2u,
// which is exact and free of cancellation as omega -> 0.  For |u| < 0.5 the
// sines and cosines of u come from their Taylor series (error < 1e-10).
template <typename T>
struct HelixT {
    T x, y;          // position at s
    T cm, sm;        // cos, sin of phi + u
    T cp, sp;        // cos, sin of phi' = phi + 2u
    T chord, S, dS;  // s sinc(u), sinc(u), d sinc/du
    T u;
};

__device__ __forceinline__ void sinc_terms(float u, float& su, float& cu, float& S, float& dS) {
    float au = fabsf(u);
    if (au < 0.5f) {
        float u2 = u * u;
        S = 1.0f + u2 * (-1.0f / 6.0f + u2 * (1.0f / 120.0f + u2 * (-1.0f / 5040.0f + u2 * (1.0f / 362880.0f))));
        cu = 1.0f + u2 * (-0.5f + u2 * (1.0f / 24.0f + u2 * (-1.0f / 720.0f + u2 * (1.0f / 40320.0f))));
        dS = u * (-1.0f / 3.0f + u2 * (1.0f / 30.0f + u2 * (-1.0f / 840.0f + u2 * (1.0f / 45360.0f))));
        su = u * S;
    } else {
        sincos_fit(u, &su, &cu);
        float iu = frcp(u);
        S = su * iu;
        dS = (cu - S) * iu;
    }
}

// FP64: the series only for |u| < 1e-3 (truncation below 1e-25), the
// library's sin and cos above.
__device__ __forceinline__ void sinc_terms(double u, double& su, double& cu, double& S, double& dS) {
    if (fabs(u) < 1e-3) {
        const double u2 = u * u;
        S = 1.0 + u2 * (-1.0 / 6.0 + u2 * (1.0 / 120.0 + u2 * (-1.0 / 5040.0)));
        cu = 1.0 + u2 * (-0.5 + u2 * (1.0 / 24.0 + u2 * (-1.0 / 720.0 + u2 * (1.0 / 40320.0))));
        dS = u * (-1.0 / 3.0 + u2 * (1.0 / 30.0 + u2 * (-1.0 / 840.0 + u2 * (1.0 / 45360.0))));
        su = u * S;
    } else {
        sincos(u, &su, &cu);
        S = su / u;
        dS = (cu - S) / u;
    }
}

template <typename T>
__device__ __forceinline__ void helix_at(T x, T y, T cphi, T sphi, T w, T s, HelixT<T>& h) {
    T u = T(0.5) * w * s;
    T su, cu;
    sinc_terms(u, su, cu, h.S, h.dS);
    h.u = u;
    h.chord = s * h.S;
    h.cm = cphi * cu - sphi * su;
    h.sm = sphi * cu + cphi * su;
    h.x = fma_(h.chord, h.cm, x);
    h.y = fma_(h.chord, h.sm, y);
    h.cp = h.cm * cu - h.sm * su;
    h.sp = h.sm * cu + h.cm * su;
}

// ------------------------------------------------------- cylinder crossing
// Reachability of |xy| = R from (x, y) with heading phi and curvature w,
// without dividing by w.  The track circle (centre distance d, radius rho)
// meets the layer circle iff |R - rho| <= d <= R + rho; with
// d^2 = r0^2 - 2 a'/w + rho^2, a' = x sin(phi) - y cos(phi), this reads
//   |w| (R^2 - r0^2) <= 2 (R - sign(w) a')  and  |w| (r0^2 - R^2) <= 2 (R + sign(w) a'),
// which at w = 0 reduces to the line's distance test |a'| <= R.
template <typename T>
__device__ __forceinline__ bool cylinder_reachable(T x, T y, T cphi, T sphi, T w, T R) {
    T r0sq = fma_(x, x, y * y);
    T ap = x * sphi - y * cphi;
    T sg = w >= T(0.0) ? T(1.0) : -T(1.0);
    T t = fabs(w) * (R * R - r0sq);
    return t <= T(2.0) * (R - sg * ap) && -t <= T(2.0) * (R + sg * ap);
}

// How far behind the start a surface may lie and still be the next one
// (transverse path, cm): an update can leave the state slightly beyond the
// next surface, which a short backward step then reaches.
constexpr float BACK_TOL = 1.0f;

// Straight-line path to |xy| = R: the first root beyond -BACK_TOL.  With
// b = x cos(phi) + y sin(phi) and d = R^2 - r0^2 the roots are
// -b -/+ sqrt(b^2 + d), each taken in its cancellation-free form.  *ok is
// false when no root lies beyond -BACK_TOL.
template <typename T>
__device__ __forceinline__ T line_path(T x, T y, T cphi, T sphi, T R, bool* ok) {
    T b = x * cphi + y * sphi;
    T r0sq = fma_(x, x, y * y);
    T dr2 = R * R - r0sq;
    T disc = fma_(b, b, dr2);
    T sq = sqrt_start_(fmax(disc, T(0.0)));
    T lo, hi;   // lo <= hi
    if (b >= T(0.0)) {
        lo = -(b + sq);
        hi = (b + sq) > T(0.0) ? div_(dr2, b + sq) : T(0.0);
    } else {
        lo = div_(dr2, b - sq);
        hi = sq - b;
    }
    *ok = disc >= T(0.0) && hi > -T(BACK_TOL);
    return lo > -T(BACK_TOL) ? lo : hi;
}

// Closed-form crossing of |xy| = R within half a turn, in FP32 without
// cancellation.  With b = x cos(phi) + y sin(phi), a = y cos(phi) - x sin(phi),
// d = R^2 - r0^2 and t = tan(omega s / 2), the crossing condition
// |P(s)|^2 = R^2 is the quadratic alpha c^2 + 2 b c - d = 0 in c = 2 t / omega,
// alpha = 1 + a omega - omega^2 d / 4, with roots c = d / (b +- sqrt(b^2 + alpha d));
// then s = c atan(t) / t.  Each root is a crossing with turning angle in
// (-pi, pi); the one returned is the smallest s > -BACK_TOL.  Returns false
// if none (b^2 + alpha d < 0: the circles do not meet).
__device__ __forceinline__ float atan_ratio(float t) {   // atan(t) / t
    float at = fabsf(t);
    if (at < 0.25f) {
        float t2 = t * t;
        return 1.0f + t2 * (-1.0f / 3.0f + t2 * (1.0f / 5.0f + t2 * (-1.0f / 7.0f + t2 * (1.0f / 9.0f))));
    }
    return fdiv(atanf(t), t);
}

__device__ __forceinline__ double atan_ratio(double t) {   // atan(t) / t in FP64
    if (fabs(t) < 1e-3) {
        const double t2 = t * t;
        return 1.0 + t2 * (-1.0 / 3.0 + t2 * (1.0 / 5.0 + t2 * (-1.0 / 7.0)));
    }
    return atan(t) / t;
}

template <typename T>
__device__ __forceinline__ bool closed_form_cylinder(T x, T y, T cphi, T sphi, T w, T R,
                                                     T& s_out) {
    T b = x * cphi + y * sphi;
    T a = y * cphi - x * sphi;
    T d = R * R - fma_(x, x, y * y);
    T alpha = T(1.0) + a * w - T(0.25) * w * w * d;
    T disc = fma_(b, b, alpha * d);
    if (disc < T(0.0)) return false;
    T sq = sqrt_start_(disc);
    T den[2] = {b + sq, b - sq};
    bool have = false;
    T best = T(0.0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        T s;
        if (den[k] == T(0.0)) {
            if (w == T(0.0)) continue;             // line root at infinity
            s = div_(pi_<T>(), fabs(w));            // t = +-inf: exactly half a turn
        } else {
            T c = div_(d, den[k]);
            T t = T(0.5) * w * c;
            s = c * atan_ratio(t);
        }
        if (s > -T(BACK_TOL) && (!have || s < best)) { best = s; have = true; }
    }
    s_out = best;
    return have;
}

// Newton iteration on f(s) = (r(s)^2 - R^2) / (2R) (= r - R near the root)
// from s0 (the straight-line root or a proposal).  Stops when |f| <= tol; returns false
// after max_iter helix evaluations without convergence.  h holds the last
// evaluation, at s; *ds the Newton step that evaluation calls for, f / f',
// which the caller applies to first order (finish_crossing): at grazing
// incidence f' = cos(incidence) is small, and a residual |f| <= tol still
// leaves the crossing tol / cos(incidence) away along the track.
template <typename T>
__device__ __forceinline__ bool newton_cylinder(T x, T y, T cphi, T sphi, T w, T R,
                                                T tol, int max_iter, T s0, T& s, HelixT<T>& h,
                                                int& iters, bool have_first = false, T* ds = nullptr) {
    const T invR = rcp_(R);
    const T inv2R = T(0.5) * invR;
    s = s0;
    for (int it = 0; it < max_iter; ++it) {
        if (!(have_first && it == 0)) helix_at(x, y, cphi, sphi, w, s, h);
        T f = (fma_(h.x, h.x, h.y * h.y) - R * R) * inv2R;
        iters = it + 1;
        T fp = (h.x * h.cp + h.y * h.sp) * invR;
        T step = div_(f, fp);
        if (fabs(f) <= tol) {
            if (ds) *ds = step;
            return true;
        }
        s -= step;
    }
    return false;
}

// Moves a crossing found by newton_cylinder by its last Newton step -ds, to
// first order along the track: position along (cos phi', sin phi'), phi' by
// omega times the step.  The second-order remainder, |ds|^2 / (2R), is far
// below any tolerance for |ds| <= 0.1 cm; a larger step (a track tangent to
// the surface, where the crossing itself is ill-defined) is not applied.
// Returns the step applied.
template <typename T>
__device__ __forceinline__ T finish_crossing(T w, T ds, T& s, HelixT<T>& h) {
    const T d = fabs(ds) <= T(0.1) ? ds : T(0);
    s -= d;
    h.x = fma_(-d, h.cp, h.x);
    h.y = fma_(-d, h.sp, h.y);
    const T dphi = -w * d;
    h.u = fma_(T(0.5), dphi, h.u);
    const T cp = h.cp, sp = h.sp;
    h.cp = fma_(-sp, dphi, cp);
    h.sp = fma_(cp, dphi, sp);
    return d;
}

// -------------------------------------------------------- Jacobian blocks
// Derivatives of the helix point at fixed s (omega = kq * ipt):
//   dx'/domega = (s^2/2) (sinc'(u) cos phi_m - sinc(u) sin phi_m)
//   dy'/domega = (s^2/2) (sinc'(u) sin phi_m + sinc(u) cos phi_m)
//   dx'/dphi = -chord sin phi_m,  dy'/dphi = chord cos phi_m
//   dphi'/domega = s,  dz'/dtheta = -s / sin^2 theta,  d(x', y', z', phi')/ds = (cos phi', sin phi', cot theta, omega)
// The path s*(p) to the surface adds (d state/ds) (ds*/dp)^T, with
// ds*/dp = -(dg/dp) / (dg/ds) for the surface constraint g(state(p, s)) = 0.
template <typename T>
struct JacT {
    // rows x, y, phi: columns x, y, z, ipt, phi, theta (some are structurally 0)
    T a[3][6];
    // row z: columns x, y, z, ipt, phi, theta
    T z[6];
};

// Cylinder: g = x'^2 + y'^2 - R^2, dg/ds = 2 D, D = x' cos phi' + y' sin phi'.
// ds/dx = -x'/D, ds/dy = -y'/D, ds/dphi = -(x' y - x y')/D,
// ds/dipt = -kq (x' dx'/domega + y' dy'/domega)/D, ds/dz = ds/dtheta = 0.
// dxp, dyp: the displacements x' - x and y' - y (chord cos(phi_m) and
// chord sin(phi_m) at the last helix evaluation, moved by the step
// finish_crossing applied).
template <typename T>
__device__ __forceinline__ void jacobian_cylinder(T x, T y, T w, T kq, T s, T cot,
                                                  T sinth, const HelixT<T>& h, JacT<T>& J, T dxp, T dyp) {
    T hs2 = T(0.5) * s * s;
    T dxw = hs2 * (h.dS * h.cm - h.S * h.sm);
    T dyw = hs2 * (h.dS * h.sm + h.S * h.cm);
    T iD = rcp_(h.x * h.cp + h.y * h.sp);
    T dsx = -h.x * iD;
    T dsy = -h.y * iD;
    T dsphi = -(h.x * y - x * h.y) * iD;
    T dsipt = -kq * (h.x * dxw + h.y * dyw) * iD;
    // x' row
    J.a[0][0] = fma_(h.cp, dsx, T(1.0));
    J.a[0][1] = h.cp * dsy;
    J.a[0][2] = T(0.0);
    J.a[0][3] = fma_(h.cp, dsipt, kq * dxw);
    J.a[0][4] = fma_(h.cp, dsphi, -dyp);
    J.a[0][5] = T(0.0);
    // y' row
    J.a[1][0] = h.sp * dsx;
    J.a[1][1] = fma_(h.sp, dsy, T(1.0));
    J.a[1][2] = T(0.0);
    J.a[1][3] = fma_(h.sp, dsipt, kq * dyw);
    J.a[1][4] = fma_(h.sp, dsphi, dxp);
    J.a[1][5] = T(0.0);
    // phi' row
    J.a[2][0] = w * dsx;
    J.a[2][1] = w * dsy;
    J.a[2][2] = T(0.0);
    J.a[2][3] = fma_(w, dsipt, kq * s);
    J.a[2][4] = fma_(w, dsphi, T(1.0));
    J.a[2][5] = T(0.0);
    // z' row
    J.z[0] = cot * dsx;
    J.z[1] = cot * dsy;
    J.z[2] = T(1.0);
    J.z[3] = cot * dsipt;
    J.z[4] = cot * dsphi;
    J.z[5] = -div_(s, sinth * sinth);
}

// Plane: g = z' - Z; ds/dz = -tan(theta), ds/dtheta = s / (sin cos), others 0.
// The z' row vanishes (z' = Z).
template <typename T>
__device__ __forceinline__ void jacobian_plane(T w, T kq, T s, T tanth, T sinth, T costh,
                                               const HelixT<T>& h, JacT<T>& J) {
    T hs2 = T(0.5) * s * s;
    T dxw = hs2 * (h.dS * h.cm - h.S * h.sm);
    T dyw = hs2 * (h.dS * h.sm + h.S * h.cm);
    T dsz = -tanth;
    T dsth = div_(s, sinth * costh);
    J.a[0][0] = T(1.0);  J.a[0][1] = T(0.0);  J.a[0][2] = h.cp * dsz;  J.a[0][3] = kq * dxw;
    J.a[0][4] = -h.chord * h.sm;  J.a[0][5] = h.cp * dsth;
    J.a[1][0] = T(0.0);  J.a[1][1] = T(1.0);  J.a[1][2] = h.sp * dsz;  J.a[1][3] = kq * dyw;
    J.a[1][4] = h.chord * h.cm;   J.a[1][5] = h.sp * dsth;
    J.a[2][0] = T(0.0);  J.a[2][1] = T(0.0);  J.a[2][2] = w * dsz;     J.a[2][3] = kq * s;
    J.a[2][4] = T(1.0);  J.a[2][5] = w * dsth;
    for (int k = 0; k < 6; ++k) J.z[k] = T(0.0);
}

// ------------------------------------------------- covariance transport
// C' = J C J^T on the packed covariance.  Rows ipt and theta of J are unit
// rows.  SURF 0 (cylinder): rows x, y, phi have non-zeros in columns
// x, y, ipt, phi; row z in all columns (z coefficient 1).  SURF 1 (plane):
// rows x, y, phi in all columns except (x: y), (y: x), (phi: x, y); row z = 0.
// The structural zeros are skipped at compile time through the masks.
template <int SURF, typename T>
__device__ __forceinline__ void transport(const JacT<T>& J, T* c) {
    // column masks of the x, y, phi rows
    constexpr unsigned MX = SURF == 0 ? 0b011011u : 0b111101u;   // bit k: column k used
    constexpr unsigned MY = SURF == 0 ? 0b011011u : 0b111110u;
    constexpr unsigned MP = SURF == 0 ? 0b011011u : 0b111100u;
    // rows of M = J C for the transformed rows x(0), y(1), phi(4), z(2)
    T M0[6], M1[6], M4[6], M2[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        T m0 = T(0.), m1 = T(0.), m4 = T(0.);
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            if (MX & (1u << l)) m0 = fma_(J.a[0][l], c[I21(l, k)], m0);
            if (MY & (1u << l)) m1 = fma_(J.a[1][l], c[I21(l, k)], m1);
            if (MP & (1u << l)) m4 = fma_(J.a[2][l], c[I21(l, k)], m4);
        }
        M0[k] = m0; M1[k] = m1; M4[k] = m4;
        if (SURF == 0) {
            T m2 = c[I21(2, k)];
#pragma unroll
            for (int l = 0; l < 6; ++l)
                if (l != 2) m2 = fma_(J.z[l], c[I21(l, k)], m2);
            M2[k] = m2;
        }
    }
    // new rows: r(i) returns the row of M for transformed index i; rows 3, 5 are C's
    auto Mrow = [&](int i, int k) -> T {
        switch (i) {
            case 0: return M0[k];
            case 1: return M1[k];
            case 2: return SURF == 0 ? M2[k] : T(0.0);
            case 4: return M4[k];
            default: return c[I21(i, k)];
        }
    };
    auto dotJ = [&](int i, int j) -> T {   // (M J^T)_{ij} = sum_k M_ik J_jk
        if (j == 3 || j == 5) return Mrow(i, j);
        if (j == 2) {
            if (SURF == 1) return T(0.0);
            T a = Mrow(i, 2);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if (k != 2) a = fma_(Mrow(i, k), J.z[k], a);
            return a;
        }
        const unsigned m = j == 0 ? MX : (j == 1 ? MY : MP);
        const int r = j == 0 ? 0 : (j == 1 ? 1 : 2);
        T a = T(0.);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (m & (1u << k)) a = fma_(Mrow(i, k), J.a[r][k], a);
        return a;
    };
    T n[21];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) n[I21(i, j)] = dotJ(i, j);
#pragma unroll
    for (int k = 0; k < 21; ++k) c[k] = n[k];
}

// ----------------------------------------------------------- Kalman update
// 3x3 symmetric inverse through S = L D L^T (L unit lower triangular),
// S^-1 = L^-T D^-1 L^-1, with the positive-definiteness test on the pivots:
//   d0 = S00 > 0,  d1 = S11 - S10^2 / S00 > tau S11,  d2 > tau S22.
// Each pivot comes from one subtraction from a diagonal element, so it keeps
// its accuracy when S is ill-conditioned -- a large prior variance along the
// surface (a track crossing at a shallow angle) against a precise hit --
// where the cofactor form loses digits twice, in the 2x2 minors and again in
// the determinant, and the Joseph update then turns that error of S^-1 into
// one of the posterior covariance larger by the ratio of prior to posterior
// variance.
template <typename T>
__device__ __forceinline__ bool inv3_spd(const T s[6], T inv[6], T tau) {
    // s: packed (00, 10, 11, 20, 21, 22)
    const T d0 = s[0];
    const T i0 = rcp_(d0);
    const T l10 = s[1] * i0, l20 = s[3] * i0;
    const T d1 = fma_(-l10, s[1], s[2]);
    const T e21 = fma_(-l20, s[1], s[4]);
    const T i1 = rcp_(d1);
    const T l21 = e21 * i1;
    const T d2 = fma_(-l21, e21, fma_(-l20, s[3], s[5]));
    const bool ok = (d0 > T(0)) && (d1 > tau * s[2]) && (d2 > tau * s[5]);
    if (!ok) return false;
    const T i2 = rcp_(d2);
    // L^-1 = [[1, 0, 0], [-l10, 1, 0], [l10 l21 - l20, -l21, 1]]
    const T m20 = fma_(l10, l21, -l20);
    const T t20 = m20 * i2;                  // (S^-1)_20
    const T t21 = -l21 * i2;                 // (S^-1)_21
    const T v10 = -l10 * i1;
    inv[5] = i2;
    inv[4] = t21;
    inv[3] = t20;
    inv[2] = fma_(-l21, t21, i1);
    inv[1] = fma_(-l21, t20, v10);
    inv[0] = fma_(m20, t20, fma_(-l10, v10, i0));
    return true;
}

// Full update in FP64 for an ill-conditioned S (the FP32 test failed).
// When S is ill-conditioned the update shrinks some variances by orders of
// magnitude in one step, and FP32 products of the gain would lose the digits
// an FP64 inverse keeps; so this path also forms the gain and the Joseph
// covariance in FP64.  Kept out of line, with loops over small arrays, so its
// registers do not weigh on the FP32 path that runs almost always.
struct Fp64Io {
    double p[6];   // the state's parameters with their low parts
    float c[21], m[3], V[6], chi2;
};

__device__ __noinline__ uint32_t kalman_update_fp64(Fp64Io* io, float chi2_cut) {
    double* p = io->p;
    float* c = io->c;
    const float* m = io->m;
    const float* V = io->V;
    float* chi2 = &io->chi2;
    double C[6][6], Vd[3][3], S[6], Si[6], K[6][3], A[6][6], M[6][6];
#pragma unroll 1
    for (int i = 0; i < 6; ++i)
#pragma unroll 1
        for (int j = 0; j < 6; ++j) C[i][j] = (double)c[I21(i, j)];
#pragma unroll 1
    for (int i = 0; i < 3; ++i)
#pragma unroll 1
        for (int j = 0; j < 3; ++j) Vd[i][j] = (double)V[I21(i, j)];
    S[0] = C[0][0] + Vd[0][0]; S[1] = C[1][0] + Vd[1][0]; S[2] = C[1][1] + Vd[1][1];
    S[3] = C[2][0] + Vd[2][0]; S[4] = C[2][1] + Vd[2][1]; S[5] = C[2][2] + Vd[2][2];
    if (!inv3_spd<double>(S, Si, PD_TAU64)) return ST_S_NOT_PD;
    double Sm[3][3] = {{Si[0], Si[1], Si[3]}, {Si[1], Si[2], Si[4]}, {Si[3], Si[4], Si[5]}};
    double r[3], w[3], c2 = 0.0;
#pragma unroll 1
    for (int i = 0; i < 3; ++i) r[i] = (double)m[i] - p[i];
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
        w[i] = Sm[i][0] * r[0] + Sm[i][1] * r[1] + Sm[i][2] * r[2];
        c2 += r[i] * w[i];
    }
    if (chi2_cut > 0.0f && c2 > (double)chi2_cut) return ST_CHI2_CUT;
    *chi2 = (float)c2;
#pragma unroll 1
    for (int i = 0; i < 6; ++i) {
        double dp = 0.0;
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
            K[i][j] = C[i][0] * Sm[0][j] + C[i][1] * Sm[1][j] + C[i][2] * Sm[2][j];
            dp += C[i][j] * w[j];
        }
        p[i] += dp;
    }
#pragma unroll 1
    for (int i = 0; i < 6; ++i)
#pragma unroll 1
        for (int j = 0; j < 6; ++j) A[i][j] = (i == j ? 1.0 : 0.0) - (j < 3 ? K[i][j] : 0.0);
#pragma unroll 1
    for (int i = 0; i < 6; ++i)
#pragma unroll 1
        for (int l = 0; l < 6; ++l) {
            double a = 0.0;
#pragma unroll 1
            for (int k = 0; k < 6; ++k) a += A[i][k] * C[k][l];
            M[i][l] = a;
        }
#pragma unroll 1
    for (int i = 0; i < 6; ++i)
#pragma unroll 1
        for (int l = 0; l <= i; ++l) {
            double a = 0.0;
#pragma unroll 1
            for (int k = 0; k < 6; ++k) a += M[i][k] * A[l][k];
#pragma unroll 1
            for (int j = 0; j < 3; ++j)
#pragma unroll 1
                for (int k = 0; k < 3; ++k) a += K[i][j] * Vd[j][k] * K[l][k];
            c[I21(i, l)] = (float)a;
        }
    return 0;
}

// Update on a cylinder in the hit's (r-phi, z) frame.  With (c, s) the
// hit's direction in the transverse plane only the two coordinates along the
// surface are measured: u = -s x + c y (u_hit = 0) and z, i.e.
//   H = [[-s, c, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0]],  V2 = R V R^T,
//   R = [[-s, c, 0], [0, 0, 1]];
// then S = H C' H^T + V2 (2x2), K = C' H^T S^-1 (6x2), p+ = p' + K r,
// chi2 = r^T S^-1 r, and the Joseph covariance, evaluated as
// C+ = M + (K V2 - M H^T) K^T with M = A C' = C' - K (C' H^T)^T, as in
// kalman_update_surf.  Same skip rules, fallback modes and zero-gain trick
// as there.
template <typename T>
__device__ __forceinline__ uint32_t kalman_update_2d(StateT<T>& st, const T m[3], const T V[6],
                                                     const Params& P, T& chi2, uint32_t& flags);

struct Fp64Io2 {
    double p[6];   // the state's parameters with their low parts
    float c[21], m[3], V[6], chi2;
};

// FP64 inverse of the 2x2 S (fallback mode 1), out of line like the full
// FP64 update: inline, its double divisions would raise the register count
// of the whole kernel.
struct Inv2Io {
    float s00, s01, s11, i00, i01, i11;
};
__device__ __noinline__ bool inv2_fp64(Inv2Io* io) {
    const double d00 = io->s00, d01 = io->s01, d11 = io->s11;
    const double dd = d00 * d11 - d01 * d01;
    if (!(d00 > 0.0 && dd > PD_TAU64 * d00 * d11)) return false;
    io->i00 = (float)(d11 / dd);
    io->i01 = (float)(-d01 / dd);
    io->i11 = (float)(d00 / dd);
    return true;
}
__device__ __noinline__ uint32_t kalman_update_2d_fp64(Fp64Io2* io, float chi2_cut);

template <typename T>
__device__ __forceinline__ uint32_t kalman_update_2d(StateT<T>& st, const T m[3], const T V[6],
                                                     const Params& P, T& chi2, uint32_t& flags) {
    constexpr bool F32 = sizeof(T) == sizeof(float);
    T* c = st.c;
    const T rh2 = fma_(m[0], m[0], m[1] * m[1]);
    const T irh = rcp_(sqrt_start_(rh2));
    const T ch = m[0] * irh, sh = m[1] * irh;
    const T v00 = fma_(sh * sh, V[0], fma_(T(-2) * sh * ch, V[1], ch * ch * V[2]));
    const T v01 = fma_(-sh, V[3], ch * V[4]);
    const T v11 = V[5];
    // S = H C' H^T + V2 from the position block alone; P = C' H^T (all six
    // rows) is formed only after the rare FP64 branch, so that it is not
    // live across that call
    const T q0 = fma_(-sh, c[I21(0, 0)], ch * c[I21(0, 1)]);
    const T q1 = fma_(-sh, c[I21(1, 0)], ch * c[I21(1, 1)]);
    const T S00 = fma_(-sh, q0, fma_(ch, q1, v00));
    const T S01 = fma_(-sh, c[I21(2, 0)], ch * c[I21(2, 1)]) + v01;
    const T S11 = c[I21(2, 2)] + v11;
    const T det = fma_(S00, S11, -S01 * S01);
    const T tau = F32 ? T(PD_TAU32) : T(PD_TAU_F64_FIT);
    const bool pd = S00 > T(0) && det > tau * S00 * S11;
    T id = rcp_(det);
    T Si00 = S11 * id, Si01 = -S01 * id, Si11 = S00 * id;
    uint32_t res = 0;
    bool done = false;
    if constexpr (!F32) {
        if (!pd) res = ST_S_NOT_PD;
    } else if (P.fp64_fallback == 2 || !pd) {
        if (!P.fp64_fallback) {
            res = ST_S_NOT_PD;
        } else {
            flags |= ST_FP64_FALLBACK;
            if (P.fp64_fallback != 1) {
                Fp64Io2 io;
#pragma unroll
                for (int k = 0; k < 6; ++k) io.p[k] = (double)st.p[k] + (double)st.lo[k];
#pragma unroll
                for (int k = 0; k < 21; ++k) io.c[k] = (float)st.c[k];
#pragma unroll
                for (int k = 0; k < 3; ++k) io.m[k] = (float)m[k];
#pragma unroll
                for (int k = 0; k < 6; ++k) io.V[k] = (float)V[k];
                io.chi2 = (float)chi2;
                res = kalman_update_2d_fp64(&io, P.chi2_cut);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    st.p[k] = (float)io.p[k];
                    st.lo[k] = k == 3 ? T(0) : (T)(io.p[k] - (double)st.p[k]);
                }
#pragma unroll
                for (int k = 0; k < 21; ++k) st.c[k] = io.c[k];
                chi2 = io.chi2;
                done = true;
            } else {
                Inv2Io io{(float)S00, (float)S01, (float)S11, 0.0f, 0.0f, 0.0f};
                if (!inv2_fp64(&io)) res = ST_S_NOT_PD;
                Si00 = io.i00;
                Si01 = io.i01;
                Si11 = io.i11;
            }
        }
    }
    // P = C' H^T: column 0 = -s C'(:,x) + c C'(:,y), column 1 = C'(:,z)
    T P0[6], P1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        P0[i] = fma_(-sh, c[I21(i, 0)], ch * c[I21(i, 1)]);
        P1[i] = c[I21(i, 2)];
    }
    // residual in the hit frame from the position differences
    const T dx = residual_of(st, 0, m[0]), dy = residual_of(st, 1, m[1]);
    const T r0 = fma_(-sh, dx, ch * dy);
    const T r1 = residual_of(st, 2, m[2]);
    T w0 = fma_(Si00, r0, Si01 * r1);
    T w1 = fma_(Si01, r0, Si11 * r1);
    const T c2 = fma_(r0, w0, r1 * w1);
    if (res == 0 && !done && P.chi2_cut > 0.0f && c2 > T(P.chi2_cut)) res = ST_CHI2_CUT;
    const bool apply = res == 0 && !done;
    if (apply) chi2 = c2;
    w0 = apply ? w0 : T(0);
    w1 = apply ? w1 : T(0);
    Si00 = apply ? Si00 : T(0);
    Si01 = apply ? Si01 : T(0);
    Si11 = apply ? Si11 : T(0);
    T K0[6], K1[6], KV0[6], KV1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        K0[i] = fma_(P0[i], Si00, P1[i] * Si01);
        K1[i] = fma_(P0[i], Si01, P1[i] * Si11);
        KV0[i] = fma_(K0[i], v00, K1[i] * v01);
        KV1[i] = fma_(K0[i], v01, K1[i] * v11);
        const T dp = fma_(P0[i], w0, P1[i] * w1);
        if (i == 3) st.p[i] += dp;
        else add_to(st, i, dp);
    }
    // M = A C' = C' - K P^T (entries (i, l) with l <= i, and l < 3)
    T M[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int l = 0; l < 6; ++l)
            if (l <= i || l < 3) M[i][l] = fma_(-K0[i], P0[l], fma_(-K1[i], P1[l], c[I21(i, l)]));
    T D0[6], D1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        D0[i] = KV0[i] - fma_(-sh, M[i][0], ch * M[i][1]);
        D1[i] = KV1[i] - M[i][2];
    }
    T n[21];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int l = 0; l <= i; ++l) n[I21(i, l)] = fma_(D0[i], K0[l], fma_(D1[i], K1[l], M[i][l]));
#pragma unroll
    for (int k = 0; k < 21; ++k) c[k] = n[k];
    return res;
}

// The 3D-hit update taken in the surface frame.  After the transport the
// state lies on the surface, so the position block of C' has the surface
// normal n as a null direction: C' H^T has no component along n.  With the
// orthonormal frame (t1, t2, n) of the crossing point -- cylinder: t1 =
// (-s, c, 0), t2 = z, n = (c, s, 0), (c, s) = (x, y) / r; plane z = Z: t1 = x,
// t2 = y, n = z -- the 3x3 innovation covariance is
//   S = [[A + Vtt, Vtn], [Vtn^T, Vnn]],  A = [t1 t2]^T C'_pos [t1 t2],
// and block elimination of its n row (a Schur complement of Vnn) gives the
// same update as the 3x3 one in exact arithmetic:
//   V^ = Vtt - Vtn Vtn^T / Vnn,  r^ = r_t - Vtn r_n / Vnn,
//   S^ = A + V^ (2x2),  K = C' H^T S^-1 = P S^^-1 [I | -Vtn / Vnn],
//   p+ = p' + P S^^-1 r^,  C+ = C' - P S^^-1 P^T (Joseph form below),
//   chi2 = r^T S^-1 r = r^^T S^^-1 r^ + r_n^2 / Vnn   (3 degrees of freedom),
// with P = C' [t1 t2] (6x2).  This is the 2x2 update of kalman_update_2d in
// the crossing point's frame with the measurement covariance and residual
// corrected for the normal component, at about two thirds of the cost of
// the 3x3 algebra.  KIND 0: cylinder, 1: plane, 2: chosen per lane by
// `kind` (kernels whose lanes meet both in one row share one update).
//
// The Joseph form, C+ = A C' A^T + K V^ K^T with A = I - K H, is evaluated
// as M + (K V^ - M H^T) K^T, M = A C' = C' - K P^T: at the optimal gain
// M H^T = K V^ exactly, so K V^ - M H^T holds only the rounding residual the
// Joseph form exists to absorb, and forming it first subtracts the two
// nearly equal terms exactly instead of carrying both through every element.
// The posterior keeps close to FP32 relative accuracy even when the update
// shrinks C' by orders of magnitude.
//
// When the FP32 positive-definiteness test (the pivots of S^, and V_nn > 0)
// fails: fp64_fallback 3 runs the whole 3x3 update in FP64
// (kalman_update_fp64), 1 inverts S^ in FP64 and continues in FP32, 0 skips
// the update; mode 2 runs the FP64 update for every surface (testing).
// Returns 0, or ST_S_NOT_PD / ST_CHI2_CUT when the update is skipped;
// ST_FP64_FALLBACK is OR-ed into *flags when an FP64 path ran.
//
// The FP32 arithmetic has no branch: a lane whose update is skipped (or was
// done by the FP64 path) runs it with S^-1 and w set to zero, so that K = 0
// and every FMA below returns its accumulator unchanged -- p and C come out
// bit for bit as they went in.  Branching around it instead makes the
// compiler copy the whole state into merge registers on every layer.
template <typename T, int KIND>
__device__ __forceinline__ uint32_t kalman_update_surf(StateT<T>& st, const T m[3], const T V[6],
                                                       const Params& P, T& chi2, uint32_t& flags,
                                                       int kind = KIND) {
    constexpr bool F32 = sizeof(T) == sizeof(float);
    T* c = st.c;
    // frame: t1 = (a0, a1, 0), t2 = (0, b1, b2), n = (n0, n1, n2)
    T a0, a1, b1, b2, n0, n1, n2;
    if constexpr (KIND == 1) {
        a0 = T(1); a1 = T(0); b1 = T(1); b2 = T(0); n0 = T(0); n1 = T(0); n2 = T(1);
    } else {
        const T ir = rcp_(sqrt_start_(fma_(st.p[0], st.p[0], st.p[1] * st.p[1])));
        const T cc = st.p[0] * ir, ss = st.p[1] * ir;
        if constexpr (KIND == 0) {
            a0 = -ss; a1 = cc; b1 = T(0); b2 = T(1); n0 = cc; n1 = ss; n2 = T(0);
        } else {
            const bool pl = kind == 1;
            a0 = pl ? T(1) : -ss; a1 = pl ? T(0) : cc;
            b1 = pl ? T(1) : T(0); b2 = pl ? T(0) : T(1);
            n0 = pl ? T(0) : cc; n1 = pl ? T(0) : ss; n2 = pl ? T(1) : T(0);
        }
    }
    // projections of a 3-vector on t1, t2, n (structural zeros folded)
    auto on_t1 = [&](T vx, T vy, T vz) -> T {
        if constexpr (KIND == 1) return vx;
        else return fma_(a0, vx, a1 * vy);
    };
    auto on_t2 = [&](T vx, T vy, T vz) -> T {
        if constexpr (KIND == 0) return vz;
        else if constexpr (KIND == 1) return vy;
        else return fma_(b1, vy, b2 * vz);
    };
    auto on_n = [&](T vx, T vy, T vz) -> T {
        if constexpr (KIND == 0) return fma_(n0, vx, n1 * vy);
        else if constexpr (KIND == 1) return vz;
        else return fma_(n0, vx, fma_(n1, vy, n2 * vz));
    };
    // V t1, V t2, V n (columns of the 3x3 V), then the frame blocks
    const T Vt1x = on_t1(V[0], V[1], V[3]), Vt1y = on_t1(V[1], V[2], V[4]), Vt1z = on_t1(V[3], V[4], V[5]);
    const T Vt2x = on_t2(V[0], V[1], V[3]), Vt2y = on_t2(V[1], V[2], V[4]), Vt2z = on_t2(V[3], V[4], V[5]);
    const T vtt00 = on_t1(Vt1x, Vt1y, Vt1z);
    const T vtt01 = on_t2(Vt1x, Vt1y, Vt1z);
    const T vtt11 = on_t2(Vt2x, Vt2y, Vt2z);
    const T vtn0 = on_n(Vt1x, Vt1y, Vt1z);
    const T vtn1 = on_n(Vt2x, Vt2y, Vt2z);
    const T vnn = on_n(on_n(V[0], V[1], V[3]), on_n(V[1], V[2], V[4]), on_n(V[3], V[4], V[5]));
    const T ivnn = rcp_(vnn);
    const T g0 = vtn0 * ivnn, g1 = vtn1 * ivnn;
    const T v00 = fma_(-g0, vtn0, vtt00);
    const T v01 = fma_(-g0, vtn1, vtt01);
    const T v11 = fma_(-g1, vtn1, vtt11);
    // P = C' [t1 t2]: the rows' position parts projected
    T P0[6], P1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        P0[i] = on_t1(c[I21(i, 0)], c[I21(i, 1)], c[I21(i, 2)]);
        P1[i] = on_t2(c[I21(i, 0)], c[I21(i, 1)], c[I21(i, 2)]);
    }
    const T S00 = on_t1(P0[0], P0[1], P0[2]) + v00;
    const T S01 = on_t2(P0[0], P0[1], P0[2]) + v01;
    const T S11 = on_t2(P1[0], P1[1], P1[2]) + v11;
    const T det = fma_(S00, S11, -S01 * S01);
    const T tau = F32 ? T(PD_TAU32) : T(PD_TAU_F64_FIT);
    const bool pd = vnn > T(0) && S00 > T(0) && det > tau * S00 * S11;
    T id = rcp_(det);
    T Si00 = S11 * id, Si01 = -S01 * id, Si11 = S00 * id;
    uint32_t res = 0;
    bool done = false;
    if constexpr (!F32) {
        if (!pd) res = ST_S_NOT_PD;
    } else if (P.fp64_fallback == 2 || !pd) {
        if (!P.fp64_fallback) {
            res = ST_S_NOT_PD;
        } else {
            flags |= ST_FP64_FALLBACK;
            if (P.fp64_fallback != 1) {
                Fp64Io io;
#pragma unroll
                for (int k = 0; k < 6; ++k) io.p[k] = (double)st.p[k] + (double)st.lo[k];
#pragma unroll
                for (int k = 0; k < 21; ++k) io.c[k] = st.c[k];
#pragma unroll
                for (int k = 0; k < 3; ++k) io.m[k] = m[k];
#pragma unroll
                for (int k = 0; k < 6; ++k) io.V[k] = V[k];
                io.chi2 = (float)chi2;
                res = kalman_update_fp64(&io, P.chi2_cut);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    st.p[k] = (float)io.p[k];
                    st.lo[k] = k == 3 ? 0.0f : (float)(io.p[k] - (double)st.p[k]);
                }
#pragma unroll
                for (int k = 0; k < 21; ++k) st.c[k] = io.c[k];
                chi2 = io.chi2;
                done = true;
            } else {
                Inv2Io io{(float)S00, (float)S01, (float)S11, 0.0f, 0.0f, 0.0f};
                if (!(vnn > T(0)) || !inv2_fp64(&io)) res = ST_S_NOT_PD;
                Si00 = io.i00;
                Si01 = io.i01;
                Si11 = io.i11;
            }
        }
    }
    // residuals: along the surface (corrected for the normal one) and normal
    const T dx = residual_of(st, 0, m[0]), dy = residual_of(st, 1, m[1]), dz = residual_of(st, 2, m[2]);
    const T rn = on_n(dx, dy, dz);
    const T r0 = fma_(-g0, rn, on_t1(dx, dy, dz));
    const T r1 = fma_(-g1, rn, on_t2(dx, dy, dz));
    T w0 = fma_(Si00, r0, Si01 * r1);
    T w1 = fma_(Si01, r0, Si11 * r1);
    const T c2 = fma_(r0, w0, fma_(r1, w1, rn * rn * ivnn));
    if (res == 0 && !done && P.chi2_cut > 0.0f && c2 > T(P.chi2_cut)) res = ST_CHI2_CUT;
    const bool apply = res == 0 && !done;
    if (apply) chi2 = c2;
    w0 = apply ? w0 : T(0);
    w1 = apply ? w1 : T(0);
    Si00 = apply ? Si00 : T(0);
    Si01 = apply ? Si01 : T(0);
    Si11 = apply ? Si11 : T(0);
    T K0[6], K1[6], KV0[6], KV1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        K0[i] = fma_(P0[i], Si00, P1[i] * Si01);
        K1[i] = fma_(P0[i], Si01, P1[i] * Si11);
        KV0[i] = fma_(K0[i], v00, K1[i] * v01);
        KV1[i] = fma_(K0[i], v01, K1[i] * v11);
        const T dp = fma_(P0[i], w0, P1[i] * w1);
        if (i == 3) st.p[i] += dp;
        else add_to(st, i, dp);
    }
    // M = C' - K P^T (entries (i, l) with l <= i, and l < 3), D = K V^ - M [t1 t2],
    // C+ = M + D K^T: the Joseph form with the 2x2 V^
    T M[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int l = 0; l < 6; ++l)
            if (l <= i || l < 3) M[i][l] = fma_(-K0[i], P0[l], fma_(-K1[i], P1[l], c[I21(i, l)]));
    T D0[6], D1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        D0[i] = KV0[i] - on_t1(M[i][0], M[i][1], M[i][2]);
        D1[i] = KV1[i] - on_t2(M[i][0], M[i][1], M[i][2]);
    }
    T n[21];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int l = 0; l <= i; ++l) n[I21(i, l)] = fma_(D0[i], K0[l], fma_(D1[i], K1[l], M[i][l]));
#pragma unroll
    for (int k = 0; k < 21; ++k) c[k] = n[k];
    return res;
}

__device__ __noinline__ uint32_t kalman_update_2d_fp64(Fp64Io2* io, float chi2_cut) {
    StateT<double> sd;
    for (int k = 0; k < 6; ++k) sd.p[k] = io->p[k];   // already with the low parts
    for (int k = 0; k < 21; ++k) sd.c[k] = io->c[k];
    sd.q = 0.0;
    double m[3], V[6];
    for (int k = 0; k < 3; ++k) m[k] = io->m[k];
    for (int k = 0; k < 6; ++k) V[k] = io->V[k];
    Params Pd{};
    Pd.chi2_cut = chi2_cut;
    double c2 = io->chi2;
    uint32_t fl = 0;
    const uint32_t r = kalman_update_2d<double>(sd, m, V, Pd, c2, fl);
    for (int k = 0; k < 6; ++k) io->p[k] = sd.p[k];
    for (int k = 0; k < 21; ++k) io->c[k] = (float)sd.c[k];
    io->chi2 = (float)c2;
    return r;
}

// phi into (-pi, pi].  After a layer phi has moved by at most half a turn
// plus the update's correction, so one conditional 2 pi step is enough; an
// input far outside the range takes the general reduction first.
template <typename T>
__device__ __forceinline__ T wrap_phi(T a) {
    T r = a;
    if (!(fabs(r) <= T(3.0) * pi_<T>())) r = a - two_pi_<T>() * floor((a + pi_<T>()) * T(0.159154943091895336));
    r = r > pi_<T>() ? r - two_pi_<T>() : r;
    return r <= -pi_<T>() ? r + two_pi_<T>() : r;
}

// The same on the state's phi with its low part: 2 pi is subtracted in two
// parts (its float and the remainder), branch-free for the usual one step.
constexpr float TWO_PI_HI = 6.28318548202514648f;          // float(2 pi)
constexpr float TWO_PI_LO = -1.74845553146e-07f;            // 2 pi - TWO_PI_HI
template <typename T>
__device__ __forceinline__ void wrap_phi_state(StateT<T>& st) {
    if constexpr (sizeof(T) == sizeof(float)) {
        if (!(fabsf(st.p[4]) <= 3.0f * PI_F)) {           // far outside: plain reduction
            st.p[4] = wrap_phi(st.p[4] + st.lo[4]);
            st.lo[4] = 0.0f;
        }
        const float a = st.p[4];
        const float k = a > PI_F ? -1.0f : (a <= -PI_F ? 1.0f : 0.0f);
        add_to(st, 4, k * TWO_PI_HI);
        st.lo[4] = fmaf(k, TWO_PI_LO, st.lo[4]);
    } else {
        st.p[4] = wrap_phi(st.p[4]);
    }
}

template <typename T>
__device__ __forceinline__ bool finite3(const T m[3]) {
    return isfinite(m[0]) && isfinite(m[1]) && isfinite(m[2]);
}

template <typename T>
__device__ __forceinline__ bool bad_input(const StateT<T>& st) {
    bool bad = false;
#pragma unroll
    for (int i = 0; i < 6; ++i) bad |= !isfinite(st.p[i]);
#pragma unroll
    for (int i = 0; i < 21; ++i) bad |= !isfinite(st.c[i]);
    bad |= !(st.p[3] > T(0.0));
    bad |= !(st.p[5] > T(0.0) && st.p[5] < pi_<T>());
    return bad;
}

// --------------------------------------------------------- one layer step
// Cylinder of radius R.  s_start: proposed path length, or NaN for the
// straight-line start.  Returns the status flags of the layer; on success
// the state is updated and *updated set.  With UPDATE = false a step stops
// after the propagation (crossing, moved state, transported covariance) and
// *updated reports that the state was moved; the caller then finishes it
// with update_step.  A kernel whose lanes meet both kinds of surface in one
// row so runs one update for both.
struct StepOut {
    uint32_t flags;
    bool updated;
    int iters;
};

// U2D: the update in the hit's (r-phi, z) frame (kalman_update_2d), a
// compile-time choice so that each kernel holds only one update.
template <typename T, bool U2D = false, bool UPDATE = true>
__device__ __forceinline__ StepOut step_cylinder(StateT<T>& st, T R, const T m[3], const T V[6],
                                                 const Params& P, T& chi2, T tol, T s_start,
                                                 T accept_cm = T(0.0)) {
    StepOut o{0u, false, 0};
    if (!finite3(m)) { o.flags = ST_HIT_MISSING; return o; }
    T x = st.p[0], y = st.p[1];
    T sphi, cphi;
    sincos_comp(st, 4, &sphi, &cphi);
    T kq = -st.q * T(2.99792458e-3) * P.bz;
    T w = kq * st.p[3];
    if (!cylinder_reachable(x, y, cphi, sphi, w, R)) { o.flags = ST_NO_CROSSING; return o; }
    // start: the proposal, else the straight-line root; the closed form when
    // neither exists or when Newton ends outside the crossing window.  A
    // proposal is kept when its own residual |r(s0) - R| is at most
    // accept_cm (that evaluation is Newton's first); otherwise the plain
    // start is used and ML_REJECTED set.
    bool line_ok = true;
    HelixT<T> h;
    T s;
    T s0 = s_start;
    bool have_first = false;
    int pre = 0;
    if (!isnan(s_start)) {
        helix_at(x, y, cphi, sphi, w, s_start, h);
        const T f0 = (fma_(h.x, h.x, h.y * h.y) - R * R) * (T(0.5) * rcp_(R));
        have_first = fabs(f0) <= accept_cm && s_start > -T(BACK_TOL);
        if (!have_first) {
            o.flags |= ST_ML_REJECTED;
            pre = 1;
        }
    }
    if (!have_first && !(P.start_mode == 1 && closed_form_cylinder(x, y, cphi, sphi, w, R, s0))) {
        s0 = line_path(x, y, cphi, sphi, R, &line_ok);
        if (!line_ok && !closed_form_cylinder(x, y, cphi, sphi, w, R, s0)) { o.flags |= ST_NO_CROSSING; return o; }
    }
    T ds = T(0);
    bool conv = newton_cylinder(x, y, cphi, sphi, w, R, tol, P.max_iter, s0, s, h, o.iters, have_first, &ds);
    o.iters += pre;
    if (!conv || !(s > -T(BACK_TOL)) || fabs(w * s) > pi_<T>()) {
        T sc;
        if (!closed_form_cylinder(x, y, cphi, sphi, w, R, sc)) { o.flags |= ST_NO_CROSSING; return o; }
        int it2 = 0;
        conv = newton_cylinder(x, y, cphi, sphi, w, R, tol, P.max_iter, sc, s, h, it2, false, &ds);
        o.iters += it2;
        if (!conv || !(s > -T(BACK_TOL)) || fabs(w * s) > pi_<T>()) { o.flags |= ST_NEWTON_FAIL; return o; }
    }
    const T dapp = finish_crossing(w, ds, s, h);
    T sinth, costh;
    sincos_comp(st, 5, &sinth, &costh);
    T cot = div_(costh, sinth);
    // displacement of the crossing from the start, x' - x = chord cos(phi_m),
    // moved by the step finish_crossing applied
    const T dxp = fma_(-dapp, h.cp, h.chord * h.cm);
    const T dyp = fma_(-dapp, h.sp, h.chord * h.sm);
    JacT<T> J;
    jacobian_cylinder(x, y, w, kq, s, cot, sinth, h, J, dxp, dyp);
    add_to(st, 0, dxp);
    add_to(st, 1, dyp);
    add_to(st, 2, s * cot);
    add_to(st, 4, T(2.0) * h.u);
    transport<0>(J, st.c);
    if constexpr (!UPDATE) {
        o.updated = true;
        return o;
    }
    uint32_t u;
    if constexpr (U2D) u = kalman_update_2d(st, m, V, P, chi2, o.flags);
    else u = kalman_update_surf<T, 0>(st, m, V, P, chi2, o.flags);
    o.flags |= u;
    o.updated = (u == 0);
    wrap_phi_state(st);
    renormalise(st);
    return o;
}

// Plane z = Z.
template <typename T, bool UPDATE = true>
__device__ __forceinline__ StepOut step_plane(StateT<T>& st, T Z, const T m[3], const T V[6],
                                              const Params& P, T& chi2) {
    StepOut o{0u, false, 0};
    if (!finite3(m)) { o.flags = ST_HIT_MISSING; return o; }
    T sinth, costh;
    sincos_comp(st, 5, &sinth, &costh);
    T tanth = div_(sinth, costh);
    T s = residual_of(st, 2, Z) * tanth;     // ahead (or at most T(BACK_TOL) behind), within half a turn
    T kq = -st.q * T(2.99792458e-3) * P.bz;
    T w = kq * st.p[3];
    if (!(s > -T(BACK_TOL)) || !(fabs(w * s) <= pi_<T>())) { o.flags = ST_NO_CROSSING; return o; }
    T sphi, cphi;
    sincos_comp(st, 4, &sphi, &cphi);
    HelixT<T> h;
    helix_at(st.p[0], st.p[1], cphi, sphi, w, s, h);
    JacT<T> J;
    jacobian_plane(w, kq, s, tanth, sinth, costh, h, J);
    add_to(st, 0, h.chord * h.cm);
    add_to(st, 1, h.chord * h.sm);
    st.p[2] = Z;
    st.lo[2] = T(0);
    add_to(st, 4, T(2.0) * h.u);
    transport<1>(J, st.c);
    if constexpr (!UPDATE) {
        o.updated = true;
        return o;
    }
    uint32_t u = kalman_update_surf<T, 1>(st, m, V, P, chi2, o.flags);
    o.flags |= u;
    o.updated = (u == 0);
    wrap_phi_state(st);
    renormalise(st);
    return o;
}

// The update that ends a step taken with UPDATE = false (3D hit) on a
// surface of type `kind` (0 cylinder, 1 plane).
template <typename T>
__device__ __forceinline__ void update_step(StateT<T>& st, const T m[3], const T V[6], const Params& P,
                                            T& chi2, StepOut& o, int kind) {
    const uint32_t u = kalman_update_surf<T, 2>(st, m, V, P, chi2, o.flags, kind);
    o.flags |= u;
    o.updated = (u == 0);
    wrap_phi_state(st);
    renormalise(st);
}

// Newton tolerance for a cylinder of radius R: max(tol, 2 ulp(R)).
__device__ __forceinline__ float newton_tol(float tol, float R) {
    float ulp = __int_as_float(__float_as_int(fabsf(R)) & 0x7f800000) * 1.1920928955078125e-7f;
    return fmaxf(tol, 2.0f * ulp);
}
// FP64 fit: 1e-3 of the requested tolerance (1e-9 cm by default, so that
// the crossing's own error stays far below the FP32 rounding of the
// results), but at least 4 ulp(R).
__device__ __forceinline__ double newton_tol(float tol, double R) {
    const double ulp = __longlong_as_double(__double_as_longlong(fabs(R)) & 0x7ff0000000000000ll) *
                       2.220446049250313e-16;
    return fmax(1e-3 * (double)tol, 4.0 * ulp);
}

}  // namespace p2r
