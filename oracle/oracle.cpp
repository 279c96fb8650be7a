// FP64 reference implementation ("oracle") of the propagate + Kalman-update
// track fit of the p2r / p2z mini-apps (Section 2 of the paper: per track,
// per detector layer, propagate the track state to the layer, then Kalman
// update it with the layer's hit).
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code,
// header or constant table with the GPU library; it is deliberately plain
// and slow: full 6x6 matrices, textbook formulas, forward-mode dual numbers
// for the Jacobian, no blocking or fusion.
//
// The paper names the steps (propagateToR / propagatetoz, KalmanUpdate) but
// prints no formula, so every formula here is the textbook one:
//  * helix of a charged particle in a uniform field B z-hat, written with
//    the half-angle (sinc) form so it is exact at zero curvature;
//  * crossing with a cylinder |xy| = R: intersection of the track circle
//    with the layer circle (closed form); crossing with a plane z = Z:
//    s = (Z - z) tan(theta); in both cases the next crossing along the
//    motion, a surface at most 1 cm behind counting as the next one;
//  * transport Jacobian J = d(state after)/d(state before), including the
//    dependence of the path length on the start state, by dual numbers;
//  * C' = J C J^T;
//  * linear Kalman update with a 3D position measurement, H = [I3 | 0],
//    Joseph-form covariance update, chi2 = r^T S^-1 r.
//
// State p = (x, y, z, 1/pT, phi, theta); charge q = +-1 separate.
// Curvature omega = -q * KAPPA * B * (1/pT) [1/cm]; s = transverse arc length.
// Covariances are packed lower-triangle row-major: idx(i,j) = i(i+1)/2 + j.
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <thread>
#include <vector>

namespace {

constexpr double KAPPA = 2.99792458e-3;   // GeV / (T cm)
constexpr double PI = 3.14159265358979323846;
constexpr double HALF_PI_F32 = 1.5707963705062866;  // float32(pi/2)

// status bits (per track, OR over layers)
constexpr uint32_t ST_NO_CROSSING = 1u << 0;
constexpr uint32_t ST_S_NOT_PD = 1u << 3;
constexpr uint32_t ST_BAD_INPUT = 1u << 4;
constexpr uint32_t ST_HIT_MISSING = 1u << 6;
constexpr uint32_t ST_CHI2_CUT = 1u << 7;
constexpr uint32_t ST_DONE = 1u << 31;

// relative pivot threshold of the positive-definiteness test of S
constexpr double PD_TAU = 1e-12;
// how far behind the start point a surface may lie and still be the next
// one (transverse path, cm): an update can leave the state slightly beyond
// the next surface
constexpr double BACK_TOL = 1.0;

// ------------------------------------------------------------ dual numbers
struct Dual {
    double v;
    double d[6];
};

inline Dual cst(double v) { Dual r; r.v = v; for (int i = 0; i < 6; ++i) r.d[i] = 0.0; return r; }
inline Dual var(double v, int k) { Dual r = cst(v); r.d[k] = 1.0; return r; }
inline double val(const Dual& a) { return a.v; }
inline double val(double a) { return a; }

inline Dual chain(const Dual& a, double f, double df) {
    Dual r; r.v = f; for (int i = 0; i < 6; ++i) r.d[i] = df * a.d[i]; return r;
}
inline Dual operator+(const Dual& a, const Dual& b) { Dual r; r.v = a.v + b.v; for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r; r.v = a.v - b.v; for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r; r.v = -a.v; for (int i = 0; i < 6; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r; r.v = a.v * b.v; for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) { Dual r; r.v = a.v / b.v; for (int i = 0; i < 6; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
inline Dual operator+(const Dual& a, double b) { return a + cst(b); }
inline Dual operator+(double a, const Dual& b) { return cst(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - cst(b); }
inline Dual operator-(double a, const Dual& b) { return cst(a) - b; }
inline Dual operator*(const Dual& a, double b) { return chain(a, a.v * b, b); }
inline Dual operator*(double a, const Dual& b) { return chain(b, a * b.v, a); }
inline Dual operator/(const Dual& a, double b) { return chain(a, a.v / b, 1.0 / b); }
inline Dual operator/(double a, const Dual& b) { return cst(a) / b; }
inline Dual sin(const Dual& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
inline Dual cos(const Dual& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
inline Dual acos(const Dual& a) { return chain(a, std::acos(a.v), -1.0 / std::sqrt(1.0 - a.v * a.v)); }
inline Dual asin(const Dual& a) { return chain(a, std::asin(a.v), 1.0 / std::sqrt(1.0 - a.v * a.v)); }
inline Dual fabs(const Dual& a) { return a.v < 0 ? -a : a; }
inline Dual atan2(const Dual& y, const Dual& x) {
    double den = x.v * x.v + y.v * y.v;
    Dual r; r.v = std::atan2(y.v, x.v);
    for (int i = 0; i < 6; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / den;
    return r;
}
using std::sin; using std::cos; using std::sqrt; using std::acos; using std::asin; using std::atan2; using std::fabs;

// ------------------------------------------- FP32 rounding (measurement)
// The conditioning-measurement mode of fit_one (round32 > 0) redoes the fit
// as an FP32 implementation would, rounding values to FP32.  mode 1: round
// to nearest.  mode k >= 2: random rounding -- each value goes to one of
// its two neighbouring FP32 numbers with equal probability, drawn from a
// splitmix64 stream seeded by k and the track -- the random-rounding
// arithmetic of the CESTAC method (Vignes): the spread of the results over
// a few such runs estimates how many of their digits FP32 rounding leaves.
struct Rounder {
    int mode;
    uint64_t state;
    uint64_t next() {                      // splitmix64 (Steele, Lea, Flood 2014)
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }   // [0, 1)
    double operator()(double v) {
        const float f = (float)v;
        if (mode == 1 || !std::isfinite(v) || (double)f == v) return f;
        const float g = (double)f < v ? std::nextafter(f, INFINITY) : std::nextafter(f, -INFINITY);
        return (next() >> 63) ? f : g;
    }
};
inline double rr(Rounder* rd, double v) { return rd ? (*rd)(v) : v; }

// a constant of the arithmetic type in use (zero derivative for duals)
template <class T> inline T mk(double v) { return T(v); }
template <> inline Dual mk<Dual>(double v) { return cst(v); }

// sin(u)/u, with its Taylor series near 0 so that u = 0 is exact
template <class T> T sinc(const T& u) {
    if (std::fabs(val(u)) > 1e-4) return sin(u) / u;
    T u2 = u * u;
    return 1.0 - u2 * (1.0 / 6.0) + u2 * u2 * (1.0 / 120.0);
}

// ---------------------------------------------------------------- O1: helix
template <class T>
void helix(const T p[6], double q, double bz, const T& s, T out[6]) {
    T w = (-q * KAPPA * bz) * p[3];
    T u = w * s * 0.5;
    T chord = s * sinc(u);
    T phm = p[4] + u;
    out[0] = p[0] + chord * cos(phm);
    out[1] = p[1] + chord * sin(phm);
    out[2] = p[2] + s * cos(p[5]) / sin(p[5]);
    out[3] = p[3];
    out[4] = p[4] + w * s;
    out[5] = p[5];
}

// ------------------------------------------------- O2: crossing a cylinder
// The next crossing of x(s)^2 + y(s)^2 = R^2 along the direction of motion.
// Candidates are the (at most two) crossings within half a turn of the
// start, either way (heading change in (-pi, pi]); the crossing is the
// candidate with the smallest s > -BACK_TOL.  Returns false if there is none
// (in particular when the track circle and the layer circle do not meet).  For a state inside an outer layer and moving out
// this is the first forward crossing; a state that the previous update left
// slightly beyond the layer is taken back to it.
template <class T>
bool cross_cylinder(const T p[6], double q, double bz, double R, T* s_out) {
    const T& x = p[0]; const T& y = p[1]; const T& phi = p[4];
    T w = (-q * KAPPA * bz) * p[3];
    if (val(w) == 0.0) {  // straight line: |(x,y) + s (cos phi, sin phi)| = R
        T b = x * cos(phi) + y * sin(phi);
        T c = x * x + y * y - R * R;
        T disc = b * b - c;
        if (val(disc) < 0.0) return false;
        T sm = -b - sqrt(disc);
        T sp = -b + sqrt(disc);
        if (val(sm) > -BACK_TOL) { *s_out = sm; return true; }
        if (val(sp) > -BACK_TOL) { *s_out = sp; return true; }
        return false;
    }
    // track circle: centre c, radius rho; P(s) - c = (sin phi', -cos phi')/omega
    T rho = 1.0 / fabs(w);
    T cx = x - sin(phi) / w;
    T cy = y + cos(phi) / w;
    T d = sqrt(cx * cx + cy * cy);
    // d^2 - rho^2 = r0^2 - 2 (x sin phi - y cos phi) / omega, free of cancellation
    T e = x * x + y * y - 2.0 * (x * sin(phi) - y * cos(phi)) / w;
    T dmr = e / (d + rho);                       // d - rho
    if (!(std::fabs(val(dmr)) <= R && R <= val(d) + val(rho))) return false;
    // |P|^2 = d^2 + rho^2 + 2 rho d cos(gamma) = R^2, gamma = angle between P - c and c,
    // so cos(gamma) = A = (R^2 - d^2 - rho^2) / (2 rho d); with 1 + A = (R^2 - (d-rho)^2) / (2 rho d) and
    // 1 - A = ((d+rho)^2 - R^2) / (2 rho d), gamma is taken from the
    // half-angle forms, which stay accurate when A is near -1 or +1.
    T den = 2.0 * rho * d;
    T onepA = (R * R - dmr * dmr) / den;
    T onemA = ((d + rho) * (d + rho) - R * R) / den;
    T gamma;
    if (val(onepA) < val(onemA)) {
        T h = onepA * 0.5;
        if (val(h) < 0.0) h = mk<T>(0.0);
        gamma = 2.0 * acos(sqrt(h));
    } else {
        T h = onemA * 0.5;
        if (val(h) < 0.0) h = mk<T>(0.0);
        gamma = 2.0 * asin(sqrt(h));
    }
    // the direction of P - c is beta +- gamma, beta = direction of c
    T beta = atan2(cy, cx);
    double sgn = val(w) > 0 ? 1.0 : -1.0;
    T best = mk<T>(0.0);
    bool have = false;
    for (int k = 0; k < 2; ++k) {
        T psi = k == 0 ? beta + gamma : beta - gamma;
        T dphi = psi + sgn * (0.5 * PI) - phi;     // heading change to the crossing
        // the crossing within half a turn: heading change in (-pi, pi]
        double turns = std::floor((val(dphi) + PI) / (2.0 * PI));
        dphi = dphi - turns * (2.0 * PI);
        if (val(dphi) == -PI) dphi = dphi + 2.0 * PI;
        T s = dphi / w;
        if (!(val(s) > -BACK_TOL)) continue;
        if (!have || val(s) < val(best)) { best = s; have = true; }
    }
    if (!have) return false;
    *s_out = best;
    return true;
}

// ---------------------------------------------------- O3: crossing a plane
template <class T>
bool cross_plane(const T p[6], double q, double bz, double Z, T* s_out) {
    // s = (Z - z) tan(theta); the plane must lie ahead (or at most BACK_TOL
    // behind) and within half a turn, as for cylinders
    double ct = std::cos(val(p[5]));
    if (ct == 0.0) return false;
    T s = (Z - p[2]) * sin(p[5]) / cos(p[5]);
    if (!(val(s) > -BACK_TOL)) return false;
    double w = -q * KAPPA * bz * val(p[3]);
    if (std::fabs(w * val(s)) > PI) return false;
    *s_out = s;
    return true;
}

template <class T>
bool path_to_surface(const T p[6], double q, double bz, int type, double v, T* s) {
    return type == 0 ? cross_cylinder(p, q, bz, v, s) : cross_plane(p, q, bz, v, s);
}

// Propagate p to the surface; fills the new state and (optionally) the 6x6
// Jacobian J[i*6+j] = d p'_i / d p_j and the path length.  Returns false if
// the surface is not reached.
//
// r32 (the conditioning-measurement mode of fit_one, cylinders only): an
// FP32 fit finds the crossing as a root of the constraint (r(s)^2 - R^2) / 2R
// evaluated in FP32, whose rounding error is of order FLT_EPSILON R; its
// crossing therefore lies about FLT_EPSILON R / cos(incidence) along the
// track from the exact one (at most 0.1 cm), and its path-length
// derivatives are those of the implicit function ds/dp = -(dg/dp) / (dg/ds)
// at that point rather than at the root.  The crossing is moved by that
// amount (in random rounding, by a uniform random fraction of it either
// way) and the derivatives are formed there.
bool propagate(const double p[6], double q, double bz, int type, double v,
               double pout[6], double* J, double* s_out, Rounder* r32 = nullptr) {
    Dual pd[6], sd, od[6];
    for (int j = 0; j < 6; ++j) pd[j] = var(p[j], j);
    if (!path_to_surface(pd, q, bz, type, v, &sd)) return false;
    if (r32 && type == 0) {
        Dual h0[6];
        helix(pd, q, bz, sd, h0);
        const double D0 = h0[0].v * std::cos(h0[4].v) + h0[1].v * std::sin(h0[4].v);   // R cos(incidence)
        double shift = (double)FLT_EPSILON * v * v / std::max(std::fabs(D0), 1e-300);
        shift = std::min(shift, 0.1);
        if (r32->mode > 1) shift *= 2.0 * r32->uniform() - 1.0;   // random size and side
        Dual hf[6];
        const Dual sf = cst(sd.v + shift);
        helix(pd, q, bz, sf, hf);
        const Dual g = (hf[0] * hf[0] + hf[1] * hf[1]) * (0.5 / v);     // dg/dp at fixed s
        const double gs = (hf[0].v * std::cos(hf[4].v) + hf[1].v * std::sin(hf[4].v)) / v;   // dg/ds
        sd = sf;
        for (int j = 0; j < 6; ++j) sd.d[j] = -g.d[j] / gs;
    }
    helix(pd, q, bz, sd, od);
    for (int i = 0; i < 6; ++i) {
        pout[i] = od[i].v;
        if (J) for (int j = 0; j < 6; ++j) J[i * 6 + j] = od[i].d[j];
    }
    if (s_out) *s_out = sd.v;
    return true;
}

// --------------------------------------------------------- small matrices
inline int ix(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }
void unpack(const double* c21, double C[36]) {
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) C[i * 6 + j] = c21[ix(i, j)];
}
void pack(const double C[36], double* c21) {
    for (int i = 0; i < 6; ++i) for (int j = 0; j <= i; ++j) c21[ix(i, j)] = 0.5 * (C[i * 6 + j] + C[j * 6 + i]);
}
// generic dense product: R[m x n] = A[m x k] * B[k x n] (B given with its row stride).
// rd: operands, products and sums rounded to FP32 (the conditioning-
// measurement mode of fit_one), else FP64.
void matmul(const double* A, const double* B, double* R, int m, int k, int n, Rounder* rd = nullptr) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            if (rd) {
                double a = 0.0;
                for (int l = 0; l < k; ++l) a = (*rd)(a + (*rd)((*rd)(A[i * k + l]) * (*rd)(B[l * n + j])));
                R[i * n + j] = a;
            } else {
                double a = 0.0;
                for (int l = 0; l < k; ++l) a += A[i * k + l] * B[l * n + j];
                R[i * n + j] = a;
            }
        }
}
void transpose(const double* A, double* T, int m, int n) {
    for (int i = 0; i < m; ++i) for (int j = 0; j < n; ++j) T[j * m + i] = A[i * n + j];
}

// Cholesky of a symmetric 3x3 and its inverse.  Not PD when a pivot is
// <= PD_TAU times the corresponding diagonal element (or not finite).
template <class F>
bool inverse_spd3_t(const F S[9], F Sinv[9]) {
    F L[9] = {0};
    for (int j = 0; j < 3; ++j) {
        F dsum = S[j * 3 + j];
        for (int k = 0; k < j; ++k) dsum -= L[j * 3 + k] * L[j * 3 + k];
        if (!(dsum > PD_TAU * S[j * 3 + j]) || !std::isfinite(dsum)) return false;
        L[j * 3 + j] = std::sqrt(dsum);
        for (int i = j + 1; i < 3; ++i) {
            F a = S[i * 3 + j];
            for (int k = 0; k < j; ++k) a -= L[i * 3 + k] * L[j * 3 + k];
            L[i * 3 + j] = a / L[j * 3 + j];
        }
    }
    // S^-1 column by column: solve L L^T x = e_c
    for (int c = 0; c < 3; ++c) {
        F y[3], x[3];
        for (int i = 0; i < 3; ++i) {
            F a = (i == c) ? F(1) : F(0);
            for (int k = 0; k < i; ++k) a -= L[i * 3 + k] * y[k];
            y[i] = a / L[i * 3 + i];
        }
        for (int i = 2; i >= 0; --i) {
            F a = y[i];
            for (int k = i + 1; k < 3; ++k) a -= L[k * 3 + i] * x[k];
            x[i] = a / L[i * 3 + i];
        }
        for (int i = 0; i < 3; ++i) Sinv[i * 3 + c] = x[i];
    }
    return true;
}
// rd: every operation of the factorisation and the solves rounded to FP32
// (conditioning-measurement mode), else the FP64 routine above.
bool inverse_spd3(const double S[9], double Sinv[9], Rounder* rd = nullptr) {
    if (!rd) return inverse_spd3_t<double>(S, Sinv);
    Rounder& R = *rd;
    double L[9] = {0};
    for (int j = 0; j < 3; ++j) {
        double dsum = R(S[j * 3 + j]);
        for (int k = 0; k < j; ++k) dsum = R(dsum - R(L[j * 3 + k] * L[j * 3 + k]));
        if (!(dsum > PD_TAU * S[j * 3 + j]) || !std::isfinite(dsum)) return false;
        L[j * 3 + j] = R(std::sqrt(dsum));
        for (int i = j + 1; i < 3; ++i) {
            double a = R(S[i * 3 + j]);
            for (int k = 0; k < j; ++k) a = R(a - R(L[i * 3 + k] * L[j * 3 + k]));
            L[i * 3 + j] = R(a / L[j * 3 + j]);
        }
    }
    for (int c = 0; c < 3; ++c) {
        double y[3], x[3];
        for (int i = 0; i < 3; ++i) {
            double a = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) a = R(a - R(L[i * 3 + k] * y[k]));
            y[i] = R(a / L[i * 3 + i]);
        }
        for (int i = 2; i >= 0; --i) {
            double a = y[i];
            for (int k = i + 1; k < 3; ++k) a = R(a - R(L[k * 3 + i] * x[k]));
            x[i] = R(a / L[i * 3 + i]);
        }
        for (int i = 0; i < 3; ++i) Sinv[i * 3 + c] = x[i];
    }
    return true;
}

inline double wrap_phi(double a) {
    // into (-pi, pi]
    double r = a - 2.0 * PI * std::floor((a + PI) / (2.0 * PI));
    if (r <= -PI) r += 2.0 * PI;
    return r;
}

// FP32 rounding of an intermediate array, in the conditioning-measurement
// mode only (rd set); a no-op otherwise.
inline void rnd32(double* a, int n, Rounder* rd) {
    if (rd) for (int i = 0; i < n; ++i) a[i] = (*rd)(a[i]);
}

// ------------------------------------------------------ O6: Kalman update
// form 0: Joseph  C+ = (I-KH) C' (I-KH)^T + K V K^T
// form 1: standard C+ = (I-KH) C'
// Returns 0 updated, ST_S_NOT_PD or ST_CHI2_CUT when skipped.
uint32_t kalman_update(const double p[6], const double C[36], const double m[3], const double V21[6],
                       int form, double chi2_cut, double pout[6], double Cout[36], double* chi2,
                       Rounder* r32 = nullptr) {
    double V[9];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
        int a = i > j ? i : j, b = i > j ? j : i;
        V[i * 3 + j] = V21[a * (a + 1) / 2 + b];
    }
    double S[9], Sinv[9];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) S[i * 3 + j] = C[i * 6 + j] + V[i * 3 + j];
    rnd32(S, 9, r32);
    if (!inverse_spd3(S, Sinv, r32)) return ST_S_NOT_PD;
    rnd32(Sinv, 9, r32);
    double r[3];
    for (int i = 0; i < 3; ++i) r[i] = m[i] - p[i];
    rnd32(r, 3, r32);
    double c2 = 0.0;
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) c2 += r[i] * Sinv[i * 3 + j] * r[j];
    rnd32(&c2, 1, r32);
    if (chi2_cut > 0.0 && c2 > chi2_cut) return ST_CHI2_CUT;
    // K = C' H^T S^-1 ; C' H^T = first three columns of C'
    double PHt[18], K[18];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 3; ++j) PHt[i * 3 + j] = C[i * 6 + j];
    matmul(PHt, Sinv, K, 6, 3, 3, r32);
    rnd32(K, 18, r32);
    for (int i = 0; i < 6; ++i) {
        double a = 0.0;
        for (int j = 0; j < 3; ++j) a += K[i * 3 + j] * r[j];
        pout[i] = p[i] + a;
    }
    pout[4] = wrap_phi(pout[4]);
    // A = I - K H
    double A[36];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) {
        A[i * 6 + j] = (i == j ? 1.0 : 0.0) - (j < 3 ? K[i * 3 + j] : 0.0);
    }
    double AC[36];
    rnd32(A, 36, r32);
    matmul(A, C, AC, 6, 6, 6, r32);
    rnd32(AC, 36, r32);
    if (form == 1) {
        for (int i = 0; i < 36; ++i) Cout[i] = AC[i];
    } else {
        double At[36], ACAt[36], KV[18], Kt[18], KVKt[36];
        transpose(A, At, 6, 6);
        matmul(AC, At, ACAt, 6, 6, 6, r32);
        matmul(K, V, KV, 6, 3, 3, r32);
        rnd32(KV, 18, r32);
        transpose(K, Kt, 6, 3);
        matmul(KV, Kt, KVKt, 6, 3, 6, r32);
        for (int i = 0; i < 36; ++i) Cout[i] = ACAt[i] + KVKt[i];
        rnd32(Cout, 36, r32);
    }
    // symmetrise
    for (int i = 0; i < 6; ++i) for (int j = 0; j < i; ++j) {
        double a = 0.5 * (Cout[i * 6 + j] + Cout[j * 6 + i]);
        Cout[i * 6 + j] = Cout[j * 6 + i] = a;
    }
    *chi2 = c2;
    return 0;
}

// ------------------------------------------ O6': update in the hit's frame
// On a cylinder only the two coordinates along the surface are measured:
// with (c, s) the direction of the hit in the transverse plane,
//   u = -s x + c y   (the r-phi coordinate, u_hit = 0)   and   z,
// so H (2x6) = [[-s, c, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0]], the measurement
// covariance is V2 = R V R^T with R = [[-s, c, 0], [0, 0, 1]], and the
// update is the linear Kalman update with that H: S = H C' H^T + V2,
// K = C' H^T S^-1, p+ = p' + K r, Joseph C+ = (I-KH) C' (I-KH)^T + K V2 K^T,
// chi2 = r^T S^-1 r (two degrees of freedom).
uint32_t kalman_update_2d(const double p[6], const double C[36], const double m[3], const double V21[6],
                          double chi2_cut, double pout[6], double Cout[36], double* chi2,
                          Rounder* r32 = nullptr) {
    const double rh = std::hypot(m[0], m[1]);
    if (!(rh > 0.0)) return ST_S_NOT_PD;
    const double c = m[0] / rh, s = m[1] / rh;
    double H[12] = {0};
    H[0] = -s; H[1] = c; H[6 + 2] = 1.0;
    double V[9];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
        int a = i > j ? i : j, b = i > j ? j : i;
        V[i * 3 + j] = V21[a * (a + 1) / 2 + b];
    }
    const double R[6] = {-s, c, 0.0, 0.0, 0.0, 1.0};
    double RV[6], Rt[6], V2[4];
    matmul(R, V, RV, 2, 3, 3, r32);
    transpose(R, Rt, 2, 3);
    matmul(RV, Rt, V2, 2, 3, 2, r32);
    double Ht[12], CHt[12], S[4];
    transpose(H, Ht, 2, 6);
    matmul(C, Ht, CHt, 6, 6, 2, r32);
    matmul(H, CHt, S, 2, 6, 2, r32);
    for (int i = 0; i < 4; ++i) S[i] += V2[i];
    rnd32(S, 4, r32);
    // 2x2 Cholesky with the same pivot rule as the 3x3 one
    const double l00sq = S[0];
    if (!(l00sq > PD_TAU * S[0]) || !std::isfinite(l00sq)) return ST_S_NOT_PD;
    const double d1 = S[3] - S[2] * S[2] / S[0];
    if (!(d1 > PD_TAU * S[3]) || !std::isfinite(d1)) return ST_S_NOT_PD;
    const double det = S[0] * S[3] - S[1] * S[2];
    const double Sinv[4] = {S[3] / det, -S[1] / det, -S[2] / det, S[0] / det};
    double Hp[2], r[2];
    matmul(H, p, Hp, 2, 6, 1);
    const double mloc[2] = {-s * m[0] + c * m[1], m[2]};
    for (int i = 0; i < 2; ++i) r[i] = mloc[i] - Hp[i];
    rnd32(r, 2, r32);
    double c2 = 0.0;
    for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) c2 += r[i] * Sinv[i * 2 + j] * r[j];
    if (chi2_cut > 0.0 && c2 > chi2_cut) return ST_CHI2_CUT;
    double K[12];
    matmul(CHt, Sinv, K, 6, 2, 2, r32);
    rnd32(K, 12, r32);
    for (int i = 0; i < 6; ++i) pout[i] = p[i] + K[i * 2] * r[0] + K[i * 2 + 1] * r[1];
    pout[4] = wrap_phi(pout[4]);
    double KH[36], A[36], AC[36], At[36], ACAt[36], KV[12], Kt[12], KVKt[36];
    matmul(K, H, KH, 6, 2, 6, r32);
    for (int i = 0; i < 36; ++i) A[i] = ((i / 6) == (i % 6) ? 1.0 : 0.0) - KH[i];
    rnd32(A, 36, r32);
    matmul(A, C, AC, 6, 6, 6, r32);
    rnd32(AC, 36, r32);
    transpose(A, At, 6, 6);
    matmul(AC, At, ACAt, 6, 6, 6, r32);
    matmul(K, V2, KV, 6, 2, 2, r32);
    rnd32(KV, 12, r32);
    transpose(K, Kt, 6, 2);
    matmul(KV, Kt, KVKt, 6, 2, 6, r32);
    for (int i = 0; i < 36; ++i) Cout[i] = ACAt[i] + KVKt[i];
    rnd32(Cout, 36, r32);
    for (int i = 0; i < 6; ++i) for (int j = 0; j < i; ++j) {
        double a = 0.5 * (Cout[i * 6 + j] + Cout[j * 6 + i]);
        Cout[i * 6 + j] = Cout[j * 6 + i] = a;
    }
    *chi2 = c2;
    return 0;
}

// ------------------------------------------------- O7: the per-track fit
struct FitArgs {
    const double* par; const double* cov; const double* q;
    const int64_t* offsets; const uint8_t* stype; const double* sval;
    const double* hits; const double* hitcov;
    double bz, chi2_cut; int form; int update_2d;
    int round32;   // > 0: the conditioning-measurement mode with this rounding (see Rounder)
    double* par_out; double* cov_out; double* chi2_out; int32_t* nused_out; uint32_t* status_out;
    double* lay_par; double* lay_cov; double* lay_chi2;   // nullable per-surface dumps
};

bool bad_input(const double* p, const double* c21) {
    for (int i = 0; i < 6; ++i) if (!std::isfinite(p[i])) return true;
    for (int i = 0; i < 21; ++i) if (!std::isfinite(c21[i])) return true;
    if (!(p[3] > 0.0)) return true;
    if (!(p[5] > 0.0 && p[5] < PI)) return true;
    return false;
}

// round32 mode: the fit as an FP32 implementation of the same algorithm
// computes it -- the state and covariance stored as FP32 between steps, the
// matrix algebra of the transport (J C J^T) and of the update (S, its
// Cholesky inverse, K, I - K H, the Joseph products, K V K^T) done in FP32
// arithmetic -- with the helix and the crossing still evaluated in FP64,
// from the rounded state, except that a cylinder crossing is located as an
// FP32 root finder locates it (propagate).  The tests use the mode to
// measure how far FP32 rounding moves each track's result: the conditioning
// of that track's fit.  It is large where the update cancels most of the
// prior covariance (a track crossing its surface at a shallow angle carries
// a large variance along the surface, which one precise hit removes) and
// where the transport Jacobian is large.
void round_to_float(double* p, double* C, Rounder& rd) {
    for (int i = 0; i < 6; ++i) p[i] = rd(p[i]);
    for (int i = 0; i < 6; ++i) for (int j = 0; j <= i; ++j) C[i * 6 + j] = C[j * 6 + i] = rd(C[i * 6 + j]);
}

void fit_one(const FitArgs& a, int64_t t) {
    double p[6], C[36];
    for (int i = 0; i < 6; ++i) p[i] = a.par[t * 6 + i];
    unpack(a.cov + t * 21, C);
    Rounder rounder{a.round32, ((uint64_t)(uint32_t)a.round32 << 40) ^ (uint64_t)t};
    Rounder* rd = a.round32 > 0 ? &rounder : nullptr;
    double q = a.q[t];
    uint32_t st = 0;
    double chi2 = 0.0;
    int32_t nused = 0;
    const bool rejected = bad_input(p, a.cov + t * 21);
    if (rejected) {
        st |= ST_BAD_INPUT;
    } else {
        for (int64_t h = a.offsets[t]; h < a.offsets[t + 1]; ++h) {
            const double* m = a.hits + h * 3;
            if (a.stype[h] > 1) {
                st |= ST_BAD_INPUT;           // unknown surface type: surface skipped
            } else if (!(std::isfinite(m[0]) && std::isfinite(m[1]) && std::isfinite(m[2]))) {
                st |= ST_HIT_MISSING;
            } else {
                double pp[6], J[36];
                if (!propagate(p, q, a.bz, a.stype[h], a.sval[h], pp, J, nullptr, rd)) {
                    st |= ST_NO_CROSSING;
                } else {
                    double JC[36], Jt[36], Cp[36];
                    rnd32(J, 36, rd);
                    matmul(J, C, JC, 6, 6, 6, rd);
                    transpose(J, Jt, 6, 6);
                    matmul(JC, Jt, Cp, 6, 6, 6, rd);
                    for (int i = 0; i < 6; ++i) for (int j = 0; j < i; ++j) {
                        double v = 0.5 * (Cp[i * 6 + j] + Cp[j * 6 + i]);
                        Cp[i * 6 + j] = Cp[j * 6 + i] = v;
                    }
                    if (rd) round_to_float(pp, Cp, *rd);
                    double pu[6], Cu[36], c2 = 0.0;
                    uint32_t u = (a.update_2d && a.stype[h] == 0)
                                     ? kalman_update_2d(pp, Cp, m, a.hitcov + h * 6, a.chi2_cut, pu, Cu, &c2, rd)
                                     : kalman_update(pp, Cp, m, a.hitcov + h * 6, a.form, a.chi2_cut, pu, Cu, &c2,
                                                     rd);
                    if (u == 0) {
                        if (rd) round_to_float(pu, Cu, *rd);
                        std::memcpy(p, pu, sizeof p);
                        std::memcpy(C, Cu, sizeof C);
                        chi2 += c2;
                        ++nused;
                    } else {
                        st |= u;
                        std::memcpy(p, pp, sizeof p);
                        p[4] = wrap_phi(p[4]);
                        std::memcpy(C, Cp, sizeof C);
                    }
                }
            }
            if (a.lay_par) for (int i = 0; i < 6; ++i) a.lay_par[h * 6 + i] = p[i];
            if (a.lay_cov) pack(C, a.lay_cov + h * 21);
            if (a.lay_chi2) a.lay_chi2[h] = chi2;
        }
    }
    for (int i = 0; i < 6; ++i) a.par_out[t * 6 + i] = p[i];
    pack(C, a.cov_out + t * 21);
    if (rejected) for (int i = 0; i < 21; ++i) a.cov_out[t * 21 + i] = a.cov[t * 21 + i];
    a.chi2_out[t] = chi2;
    a.nused_out[t] = nused;
    a.status_out[t] = st | ST_DONE;
}

}  // namespace

extern "C" {

// Helix map O1 at a given transverse path length s.
void orc_helix(const double p[6], double q, double bz, double s, double out[6]) {
    helix(p, q, bz, s, out);
}

// Path length to a surface (type 0: cylinder |xy| = v; type 1: plane z = v).
// Returns 1 and writes s, or 0 if the surface is not reached.
int orc_path(const double p[6], double q, double bz, int type, double v, double* s) {
    return path_to_surface(p, q, bz, type, v, s) ? 1 : 0;
}

// Propagate to a surface: new state, Jacobian (row-major 6x6, nullable) and s.
int orc_propagate(const double p[6], double q, double bz, int type, double v,
                  double pout[6], double* J, double* s) {
    return propagate(p, q, bz, type, v, pout, J, s) ? 1 : 0;
}

// Kalman update O6 on full matrices.  form 0 Joseph, 1 standard.
// Returns the status bits of a skipped update (0 when updated).
uint32_t orc_update(const double p[6], const double C36[36], const double m[3], const double V21[6],
                    int form, double chi2_cut, double pout[6], double Cout36[36], double* chi2) {
    return kalman_update(p, C36, m, V21, form, chi2_cut, pout, Cout36, chi2);
}

// Update O6' in the hit's (r-phi, z) frame on a cylinder.
uint32_t orc_update_2d(const double p[6], const double C36[36], const double m[3], const double V21[6],
                       double chi2_cut, double pout[6], double Cout36[36], double* chi2) {
    return kalman_update_2d(p, C36, m, V21, chi2_cut, pout, Cout36, chi2);
}

// The per-track fit over a CSR list of surfaces.
//   par [n][6], cov [n][21], q [n]; offsets [n+1]; per surface h:
//   stype[h] (0 cylinder, 1 plane), sval[h] (radius or signed z),
//   hits [H][3], hitcov [H][6].  Outputs par_out [n][6], cov_out [n][21],
//   chi2_out [n], nused_out [n], status_out [n]; optional per-surface
//   states after each surface (lay_par [H][6], lay_cov [H][21], lay_chi2 [H]).
//   update_2d: cylinders take the update in the hit's (r-phi, z) frame (O6').
//   nthreads <= 0 means hardware concurrency.
void orc_fit(int64_t n, const double* par, const double* cov, const double* q,
             const int64_t* offsets, const uint8_t* stype, const double* sval,
             const double* hits, const double* hitcov, double bz, double chi2_cut, int form,
             int update_2d, int round32, int nthreads, double* par_out, double* cov_out, double* chi2_out,
             int32_t* nused_out, uint32_t* status_out,
             double* lay_par, double* lay_cov, double* lay_chi2) {
    FitArgs a{par, cov, q, offsets, stype, sval, hits, hitcov, bz, chi2_cut, form, update_2d, round32,
              par_out, cov_out, chi2_out, nused_out, status_out, lay_par, lay_cov, lay_chi2};
    int nt = nthreads > 0 ? nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
    if (nt > n) nt = (int)std::max<int64_t>(1, n);
    if (nt == 1) {
        for (int64_t t = 0; t < n; ++t) fit_one(a, t);
        return;
    }
    std::vector<std::thread> th;
    for (int k = 0; k < nt; ++k) {
        int64_t lo = n * k / nt, hi = n * (k + 1) / nt;
        th.emplace_back([&a, lo, hi] { for (int64_t t = lo; t < hi; ++t) fit_one(a, t); });
    }
    for (auto& x : th) x.join();
}

// Sign of the disk a track moves towards: +1 when theta < float32(pi/2).
double orc_disk_sign(double theta) { return theta < HALF_PI_F32 ? 1.0 : -1.0; }

}  // extern "C"
