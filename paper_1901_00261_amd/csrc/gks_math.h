// gks_math.h -- per-interface arithmetic of the compact 6th/8th-order
// gas-kinetic scheme (Zhao, Ji, Shyy, Xu, arXiv:1901.00261), written for
// gfx950 VALU.  Everything here is straight-line register code, templated on
// the arithmetic type T (double, or float in the mixed-precision path) and on
// the dimension (1 or 2).  State vectors always have four slots
// (rho, rho U, rho V, rho E); in 1-D slot 2 is identically zero.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include <cmath>
#include <utility>

#define GKS_HD __host__ __device__ __forceinline__

namespace gks {
// Multiply-adds are contracted into FMAs only within one statement, so a
// function rounds the same way wherever it is inlined (the single-lane,
// lane-pair and two-kernel forms of the batched 1-D step agree bit for bit).
#pragma clang fp contract(on)

// WENO-Z regularisation (reading of Sec. 3.3: 1e-6 reproduces Tables 3-4)
constexpr double kWenoEps = 1e-6;

template <typename T> GKS_HD T tabs(T x) { return x < T(0) ? -x : x; }

// Reciprocal.  FP32: the hardware reciprocal v_rcp_f32 on the device
// (about 1 ulp), the unit roundoff of the FP32 path anyway.  FP64 on the
// device: v_rcp_f64 refined by two Newton-Raphson steps (r += r (1 - x r)),
// within an ulp or so for the normal, finite, non-zero arguments the scheme
// divides by (densities, pressures, sound speeds, sums of positive
// indicators), at half the instructions of a correctly rounded division.
// On the host (and for any other type): a plain division.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__host__ inline float frcp(float x) { return 1.0f / x; }
__device__ __forceinline__ double drcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__host__ inline double drcp(double x) { return 1.0 / x; }
template <typename T> GKS_HD T rcp(T x) { return T(1) / x; }
template <> GKS_HD float rcp<float>(float x) { return frcp(x); }
template <> GKS_HD double rcp<double>(double x) { return drcp(x); }
template <typename T> GKS_HD T quot(T a, T b) { return a / b; }
template <> GKS_HD float quot<float>(float a, float b) { return a * frcp(b); }
template <> GKS_HD double quot<double>(double a, double b) { return a * drcp(b); }
// a * b + c, fused for float and double (so that code shared by two
// kernels rounds alike whatever the compiler would contract)
template <typename T> GKS_HD T fmadd(T a, T b, T c) { return a * b + c; }
template <> GKS_HD float fmadd<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> GKS_HD double fmadd<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The value of the other lane of a lane pair (lanes 2j and 2j + 1): a DPP
// quad permutation (1, 0, 3, 2), one VALU move per 32 bits.
__device__ __forceinline__ float pair_swap(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double x)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0xB1, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Type of the time-integration coefficients: FP64 when the point is
// evaluated in FP32 (their formulas cancel for tau_n comparable to dt).
template <typename D> using ExpT = std::conditional_t<std::is_same_v<D, float>, double, D>;

// ---------------------------------------------------------------------------
// Compact linear reconstruction at x_{i+1/2} (Sec. 3.1, printed formulas).
// w[0..3] = W_{i-1..i+2} (any common offset removed), d[0..3] = dx * W'.
// Returns the value (offset included by the caller), dx * P_x, dx^2 * P_xx.
// ---------------------------------------------------------------------------
template <typename T, int ORDER>
GKS_HD void linear_recon(const T* w, const T* d, T& v, T& vx, T& vxx)
{
    if constexpr (ORDER == 6) {
        v = (w[0] + T(299) * w[1] + T(299) * w[2] + w[3] - T(3) * d[0] + T(111) * d[1] - T(111) * d[2] + T(3) * d[3]) *
            T(1.0 / 600.0);
        vx = (T(-3) * w[0] - T(3411) * w[1] + T(3411) * w[2] + T(3) * w[3] + T(11) * d[0] - T(941) * d[1] -
              T(941) * d[2] + T(11) * d[3]) *
             T(1.0 / 1560.0);
        vxx = (-w[0] + w[1] + w[2] - w[3] + T(3) * d[0] - T(51) * d[1] + T(51) * d[2] - T(3) * d[3]) * T(1.0 / 40.0);
    } else {
        v = (T(25) * w[0] + T(185) * w[1] + T(185) * w[2] + T(25) * w[3] + T(6) * d[0] + T(102) * d[1] -
             T(102) * d[2] - T(6) * d[3]) *
            T(1.0 / 420.0);
        vx = (T(-14) * w[0] - T(270) * w[1] + T(270) * w[2] + T(14) * w[3] - T(3) * d[0] - T(99) * d[1] -
              T(99) * d[2] - T(3) * d[3]) *
             T(1.0 / 108.0);
        vxx = (T(-4) * w[0] + T(4) * w[1] + T(4) * w[2] - T(4) * w[3] - d[0] - T(9) * d[1] + T(9) * d[2] + d[3]) *
              T(0.25);
    }
}

// ---------------------------------------------------------------------------
// Compact WENO-Z, left state at x_{i+1/2} of one characteristic field
// (Sec. 3.3 and Appendix).  Candidate values: eq. (sub-stencil); candidate
// polynomial coefficients b_k = a_k dx^k: Appendix (w_6 with '+' before its
// x^4 term); smoothness indicator: the exact integral, whose (a_4 dx^4)^2
// coefficient is 87617/80640.  val: state; der: dx * derivative (weights
// applied to the candidates' derivatives at the interface).
// ---------------------------------------------------------------------------
template <typename T>
GKS_HD T beta4(T b1, T b2, T b3, T b4)
{
    return b1 * b1 + T(13.0 / 12.0) * b2 * b2 + T(1043.0 / 960.0) * b3 * b3 + T(87617.0 / 80640.0) * b4 * b4 +
           T(1.0 / 12.0) * b1 * b3 + T(7.0 / 80.0) * b2 * b4;
}
template <typename T> GKS_HD T beta2(T b1, T b2) { return b1 * b1 + T(13.0 / 12.0) * b2 * b2; }
template <typename T> GKS_HD T beta3(T b1, T b2, T b3)
{
    return b1 * b1 + T(13.0 / 12.0) * b2 * b2 + T(1043.0 / 960.0) * b3 * b3 + T(1.0 / 12.0) * b1 * b3;
}

template <typename T, int ORDER>
GKS_HD void weno_left(const T* w, const T* d, T& val, T& der)
{
    // candidate values at x_{i+1/2}
    const T c0 = (T(-7) * w[0] + T(13) * w[1] - T(4) * d[0]) * T(1.0 / 6.0);
    const T c1 = (-w[0] + T(5) * w[1] + T(2) * w[2]) * T(1.0 / 6.0); // w_1 == w_3
    const T c2 = (T(5) * w[1] + T(32) * w[2] - T(13) * w[3] + T(6) * d[3]) * T(1.0 / 24.0);
    const T c4 = (T(2) * w[1] + T(5) * w[2] - w[3]) * T(1.0 / 6.0);
    const T c5 = (T(10) * w[0] + T(19) * w[1] + w[2] + T(3) * d[0] + T(21) * d[1]) * T(1.0 / 30.0);
    const T c6 = (w[1] + T(19) * w[2] + T(10) * w[3] - T(21) * d[2] - T(3) * d[3]) * T(1.0 / 30.0);
    // Appendix polynomial coefficients (origin at x_i)
    const T a01 = T(-2) * w[0] + T(2) * w[1] - d[0];
    const T a02 = T(-2) * (w[0] - w[1] + d[0]);
    const T t11 = (T(-23) * w[0] + T(20) * w[1] + T(3) * w[2] - T(10) * d[0]) * T(1.0 / 16.0);
    const T t12 = w[0] - T(2) * w[1] + w[2];
    const T t13 = T(1.5) * (T(3) * w[0] - T(4) * w[1] + w[2] + T(2) * d[0]);
    const T a21 = (T(-31) * w[1] + T(60) * w[2] - T(29) * w[3] + T(14) * d[3]) * T(1.0 / 16.0);
    const T a22 = T(0.5) * (T(5) * w[1] - T(16) * w[2] + T(11) * w[3] - T(6) * d[3]);
    const T a23 = T(1.5) * (-w[1] + T(4) * w[2] - T(3) * w[3] + T(2) * d[3]);
    const T a31 = T(0.5) * (w[2] - w[0]);
    const T a32 = w[0] - T(2) * w[1] + w[2];
    const T a41 = T(0.5) * (T(-3) * w[1] + T(4) * w[2] - w[3]);
    const T a42 = w[1] - T(2) * w[2] + w[3];
    const T a51 = (w[0] - w[2] + T(10) * d[1]) * T(0.125);
    const T a52 = T(0.25) * (T(19) * w[0] - T(20) * w[1] + w[2] + T(6) * d[0] + T(12) * d[1]);
    const T a53 = T(-3) * (w[0] - w[2] + T(2) * d[1]);
    const T a54 = T(-6) * (T(5) * w[0] - T(4) * w[1] - w[2] + T(2) * d[0] + T(4) * d[1]);
    const T a61 = (T(-21) * w[1] + T(8) * w[2] + T(13) * w[3] - T(22) * d[2] - T(4) * d[3]) * T(0.125);
    const T a62 = T(0.25) * (T(25) * w[1] + T(28) * w[2] - T(53) * w[3] + T(60) * d[2] + T(18) * d[3]);
    const T a63 = T(-3) * (T(3) * w[1] + T(8) * w[2] - T(11) * w[3] + T(10) * d[2] + T(4) * d[3]);
    const T a64 = T(6) * (w[1] + T(4) * w[2] - T(5) * w[3] + T(4) * d[2] + T(2) * d[3]);

    const T b0 = beta2(a01, a02);
    const T b1 = beta3(t11, t12, t13); // beta_1 from the cubic w~_1
    const T b2 = beta3(a21, a22, a23);
    const T b3 = beta2(a31, a32);
    const T b4 = beta2(a41, a42);
    const T b5 = beta4(a51, a52, a53, a54);
    const T b6 = beta4(a61, a62, a63, a64);
    const T Z = tabs(T(3) * (b0 - b4) + (b4 - b3));
    const T eps = T(kWenoEps);
    T d0, d1, d2, d3, d4, d5, d6;
    if constexpr (ORDER == 6) {
        d0 = T(33.0 / 700.0); d1 = T(11.0 / 140.0); d2 = T(22.0 / 175.0); d3 = T(11.0 / 100.0);
        d4 = T(11.0 / 100.0); d5 = T(37.0 / 140.0); d6 = T(37.0 / 140.0);
    } else {
        d0 = T(3.0 / 98.0); d1 = T(5.0 / 98.0); d2 = T(4.0 / 49.0); d3 = T(7.0 / 98.0);
        d4 = T(7.0 / 98.0); d5 = T(17.0 / 49.0); d6 = T(17.0 / 49.0);
    }
    // alpha_k = d_k (1 + Z / e_k), e_k = beta_k + eps.
    const T e[7] = {b0 + eps, b1 + eps, b2 + eps, b3 + eps, b4 + eps, b5 + eps, b6 + eps};
    const T dk[7] = {d0, d1, d2, d3, d4, d5, d6};
    T al[7];
    if constexpr (std::is_same_v<T, float>) {
        // FP32: one hardware reciprocal per candidate (a product of seven
        // factors >= eps could leave the FP32 range)
#pragma unroll
        for (int k = 0; k < 7; ++k) al[k] = dk[k] * (T(1) + Z * rcp(e[k]));
    } else {
        // All seven scaled by prod_j e_j, which cancels in the normalisation:
        //   alpha'_k = d_k (e_k + Z) prod_{j != k} e_j,
        // formed with prefix and suffix products, so one division serves all.
        T pre[7], suf[7];
        pre[0] = T(1);
        suf[6] = T(1);
#pragma unroll
        for (int k = 1; k < 7; ++k) pre[k] = pre[k - 1] * e[k - 1];
#pragma unroll
        for (int k = 5; k >= 0; --k) suf[k] = suf[k + 1] * e[k + 1];
#pragma unroll
        for (int k = 0; k < 7; ++k) al[k] = dk[k] * (e[k] + Z) * (pre[k] * suf[k]);
    }
    const T invr = rcp(al[0] + al[1] + al[2] + al[3] + al[4] + al[5] + al[6]);
    const T al0 = al[0] * invr, al1 = al[1] * invr, al2 = al[2] * invr, al3 = al[3] * invr, al4 = al[4] * invr,
            al5 = al[5] * invr, al6 = al[6] * invr;
    val = al0 * c0 + (al1 + al3) * c1 + al2 * c2 + al4 * c4 + al5 * c5 + al6 * c6;
    // dx * derivative of each candidate at x = dx/2: b1 + b2/2 + b3/8 + b4/48
    const T g0 = a01 + T(0.5) * a02;
    const T g1 = a31 + T(0.5) * a32; // w_1 and w_3 are the same quadratic
    const T g2 = a21 + T(0.5) * a22 + T(0.125) * a23;
    const T g4 = a41 + T(0.5) * a42;
    const T g5 = a51 + T(0.5) * a52 + T(0.125) * a53 + T(1.0 / 48.0) * a54;
    const T g6 = a61 + T(0.5) * a62 + T(0.125) * a63 + T(1.0 / 48.0) * a64;
    der = al0 * g0 + (al1 + al3) * g1 + al2 * g2 + al4 * g4 + al5 * g5 + al6 * g6;
}

// Right state at x_{i+1/2}: the mirror image (reversed stencil, slopes
// negated, derivative negated back).
template <typename T, int ORDER>
GKS_HD void weno_right(const T* w, const T* d, T& val, T& der)
{
    const T wm[4] = {w[3], w[2], w[1], w[0]};
    const T dm[4] = {-d[3], -d[2], -d[1], -d[0]};
    T dd;
    weno_left<T, ORDER>(wm, dm, val, dd);
    der = -dd;
}

// ---------------------------------------------------------------------------
// Euler eigenvectors in the normal direction (slot 1 = normal velocity),
// closed form, from six scalars; entries are rebuilt on demand (keeps two
// 4x4 matrices out of the registers while the WENO-Z runs).  R: right
// eigenvectors as columns (acoustic-, entropy, shear (2-D), acoustic+),
// L = R^{-1}.
// ---------------------------------------------------------------------------
template <typename T, int DIM>
struct CharFrame {
    T U, V, c, H, b1, b2, ic;
    GKS_HD bool init(const T* W, T gamma)
    {
        const T rho = W[0], ir = rcp(rho);
        U = W[1] * ir;
        V = (DIM == 2) ? W[2] * ir : T(0);
        const T q2 = U * U + V * V;
        const T p = (gamma - T(1)) * (W[3] - T(0.5) * rho * q2);
        if (!(rho > T(0)) || !(p > T(0))) return false;
        c = sqrt(gamma * p * ir);
        H = (W[3] + p) * ir;
        ic = rcp(c);
        b1 = (gamma - T(1)) * ic * ic;
        b2 = T(0.5) * q2 * b1;
        return true;
    }
    // row a of L = R^{-1}
    GKS_HD void left(int a, T* l) const
    {
        if (a == 0) { l[0] = T(0.5) * (b2 + U * ic); l[1] = T(-0.5) * (b1 * U + ic); l[2] = T(-0.5) * b1 * V; l[3] = T(0.5) * b1; }
        else if (a == 1) { l[0] = T(1) - b2; l[1] = b1 * U; l[2] = b1 * V; l[3] = -b1; }
        else if (a == 2) { l[0] = -V; l[1] = T(0); l[2] = T(1); l[3] = T(0); }
        else { l[0] = T(0.5) * (b2 - U * ic); l[1] = T(-0.5) * (b1 * U - ic); l[2] = T(-0.5) * b1 * V; l[3] = T(0.5) * b1; }
    }
    // sum_a R[k][a] q[a]
    GKS_HD void right(const T* q, T* out) const
    {
        out[0] = q[0] + q[1] + q[3];
        out[1] = (U - c) * q[0] + U * q[1] + (U + c) * q[3];
        out[2] = DIM == 2 ? V * (q[0] + q[1] + q[3]) + q[2] : T(0);
        out[3] = (H - U * c) * q[0] + T(0.5) * (U * U + V * V) * q[1] + (DIM == 2 ? V * q[2] : T(0)) + (H + U * c) * q[3];
    }
};

// ---------------------------------------------------------------------------
// Tangential reconstruction at the three Gauss points y_j + s dy/2,
// s = -sqrt(3/5), 0, +sqrt(3/5), from the five row values j-2..j+2.
// kTanLin[g][k][r]: k-th derivative (per unit row width) of the quartic
// matching the five row averages; kTanCand / kTanLinW: the three quadratic
// candidates of the 5th-order WENO-Z and their linear weights at the point.
// ---------------------------------------------------------------------------
__device__ constexpr double kTanLin[3][3][5] = {
    {{-0.039252347340234653, 0.31298719532417346, 0.91083333333333338, -0.21632052865750681, 0.031752347340234653},
     {0.10539650012874084, -1.1755510018023716, 1.0069756700139283, 0.091115664864294968, -0.027936833204592497},
     {0.14364916731037083, 0.81270166537925825, -2.2999999999999998, 1.5872983346207417, -0.24364916731037084}},
    {{0.0046874999999999998, -0.060416666666666667, 1.1114583333333334, -0.060416666666666667, 0.0046874999999999998},
     {0.10416666666666667, -0.70833333333333337, 0.0, 0.70833333333333337, -0.10416666666666667},
     {-0.125, 1.5, -2.75, 1.5, -0.125}},
    {{0.031752347340234653, -0.21632052865750681, 0.91083333333333338, 0.31298719532417346, -0.039252347340234653},
     {0.027936833204592497, -0.091115664864294968, -1.0069756700139283, 1.1755510018023716, -0.10539650012874084},
     {-0.24364916731037084, 1.5872983346207417, -2.2999999999999998, 0.81270166537925825, 0.14364916731037083}}};

__device__ constexpr double kTanCand[3][3][3] = {
    // [gauss point][candidate][3 rows of that candidate]
    {{-0.16031583397703753, 0.70793000257481675, 0.45238583140222077},
     {0.22698250064370418, 0.93333333333333335, -0.16031583397703753},
     {1.6142808352644458, -0.84126333590815006, 0.22698250064370418}},
    {{-0.041666666666666664, 0.083333333333333329, 0.95833333333333337},
     {-0.041666666666666664, 1.0833333333333333, -0.041666666666666664},
     {0.95833333333333337, 0.083333333333333329, -0.041666666666666664}},
    {{0.22698250064370418, -0.84126333590815006, 1.6142808352644458},
     {-0.16031583397703753, 0.93333333333333335, 0.22698250064370418},
     {0.45238583140222077, 0.70793000257481675, -0.16031583397703753}}};

__device__ constexpr double kTanLinW[3][3] = {
    {0.24484385831693256, 0.61526717557251909, 0.13988896611054835},
    {-0.1125, 1.2250000000000001, -0.1125},
    {0.13988896611054835, 0.61526717557251909, 0.24484385831693256}};

// FP32 copies of the three tables (each entry rounded to nearest, as a
// conversion at the point of use would round it): the Gauss-point index is
// a run-time value, so the FP32 path loads its coefficients as FP32 and
// does not convert them at every use.
struct TanTabF {
    float lin[3][3][5], cand[3][3][3], linw[3][3];
};
constexpr TanTabF make_tan_tab_f()
{
    TanTabF t{};
    for (int g = 0; g < 3; ++g)
        for (int k = 0; k < 3; ++k) {
            for (int r = 0; r < 5; ++r) t.lin[g][k][r] = float(kTanLin[g][k][r]);
            for (int r = 0; r < 3; ++r) t.cand[g][k][r] = float(kTanCand[g][k][r]);
            t.linw[g][k] = float(kTanLinW[g][k]);
        }
    return t;
}
__device__ constexpr TanTabF kTanF = make_tan_tab_f();

// kTanLin[g][k][r] in type T
template <typename T> GKS_HD T tan_lin(int g, int k, int r)
{
    if constexpr (std::is_same_v<T, float>) return kTanF.lin[g][k][r];
    else return T(kTanLin[g][k][r]);
}

// 5th-order WENO-Z value at Gauss point g from rows q[0..4], as a quotient
// num / den; the centre point's negative linear weights are split into two
// positive groups (Shi, Hu, Shu, J. Comput. Phys. 175 (2002), theta = 3),
// whose two quotients are brought over one denominator.
template <typename T>
GKS_HD void tan_weno_frac(const T* q, int g, T& num, T& den)
{
    T cand[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        cand[k] = T(kTanCand[g][k][0]) * q[k] + T(kTanCand[g][k][1]) * q[k + 1] + T(kTanCand[g][k][2]) * q[k + 2];
    // Jiang-Shu indicators of the three quadratics over the centre row
    const T s0a = q[0] - T(2) * q[1] + q[2], s0b = q[0] - T(4) * q[1] + T(3) * q[2];
    const T s1a = q[1] - T(2) * q[2] + q[3], s1b = q[1] - q[3];
    const T s2a = q[2] - T(2) * q[3] + q[4], s2b = T(3) * q[2] - T(4) * q[3] + q[4];
    const T be[3] = {T(13.0 / 12.0) * s0a * s0a + T(0.25) * s0b * s0b, T(13.0 / 12.0) * s1a * s1a + T(0.25) * s1b * s1b,
                     T(13.0 / 12.0) * s2a * s2a + T(0.25) * s2b * s2b};
    const T Z = tabs(be[0] - be[2]);
    const T eps = T(kWenoEps);
    // alpha_k = gamma_k (1 + Z / e_k), e_k = beta_k + eps, scaled by e_0 e_1 e_2
    // (the scale cancels in the normalisation): gamma_k (e_k + Z) prod_{j != k} e_j
    const T e0 = be[0] + eps, e1 = be[1] + eps, e2 = be[2] + eps;
    const T r[3] = {(e0 + Z) * (e1 * e2), (e1 + Z) * (e0 * e2), (e2 + Z) * (e0 * e1)};
    if (g != 1) {
        T a[3];
        num = den = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) { a[k] = T(kTanLinW[g][k]) * r[k]; den += a[k]; }
#pragma unroll
        for (int k = 0; k < 3; ++k) num += a[k] * cand[k];
        return;
    }
    // gamma+ = (g + 3|g|)/2, gamma- = gamma+ - g; value sp vp - sm vm
    constexpr double gp0 = 0.1125, gp1 = 2.45, gp2 = 0.1125, sp = 2.675;
    constexpr double gm0 = 0.225, gm1 = 1.225, gm2 = 0.225, sm = 1.675;
    const T ap0 = T(gp0) * r[0], ap1 = T(gp1) * r[1], ap2 = T(gp2) * r[2];
    const T am0 = T(gm0) * r[0], am1 = T(gm1) * r[1], am2 = T(gm2) * r[2];
    const T np = ap0 * cand[0] + ap1 * cand[1] + ap2 * cand[2], dp = ap0 + ap1 + ap2;
    const T nm = am0 * cand[0] + am1 * cand[1] + am2 * cand[2], dm = am0 + am1 + am2;
    num = T(sp) * np * dm - T(sm) * nm * dp;
    den = dp * dm;
}

// The same value in FP32 arithmetic: each candidate's weight from one
// hardware reciprocal of (beta + eps), each group normalised by one more
// (products of three such factors could leave the FP32 range).
GKS_HD float tan_weno_f32(const float* q, int g)
{
    float cand[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        cand[k] = kTanF.cand[g][k][0] * q[k] + kTanF.cand[g][k][1] * q[k + 1] + kTanF.cand[g][k][2] * q[k + 2];
    const float s0a = q[0] - 2.0f * q[1] + q[2], s0b = q[0] - 4.0f * q[1] + 3.0f * q[2];
    const float s1a = q[1] - 2.0f * q[2] + q[3], s1b = q[1] - q[3];
    const float s2a = q[2] - 2.0f * q[3] + q[4], s2b = 3.0f * q[2] - 4.0f * q[3] + q[4];
    const float be[3] = {float(13.0 / 12.0) * s0a * s0a + 0.25f * s0b * s0b,
                         float(13.0 / 12.0) * s1a * s1a + 0.25f * s1b * s1b,
                         float(13.0 / 12.0) * s2a * s2a + 0.25f * s2b * s2b};
    const float Z = tabs(be[0] - be[2]);
    const float eps = float(kWenoEps);
    float w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k] = 1.0f + Z * rcp(be[k] + eps); // alpha_k / gamma_k
    if (g != 1) {
        const float a0 = kTanF.linw[g][0] * w[0], a1 = kTanF.linw[g][1] * w[1], a2 = kTanF.linw[g][2] * w[2];
        return (a0 * cand[0] + a1 * cand[1] + a2 * cand[2]) * rcp(a0 + a1 + a2);
    }
    // centre point: gamma+ = (g + 3|g|)/2, gamma- = gamma+ - g; value sp vp - sm vm
    const float ap0 = 0.1125f * w[0], ap1 = 2.45f * w[1], ap2 = 0.1125f * w[2];
    const float am0 = 0.225f * w[0], am1 = 1.225f * w[1], am2 = 0.225f * w[2];
    const float vp = (ap0 * cand[0] + ap1 * cand[1] + ap2 * cand[2]) * rcp(ap0 + ap1 + ap2);
    const float vm = (am0 * cand[0] + am1 * cand[1] + am2 * cand[2]) * rcp(am0 + am1 + am2);
    return 2.675f * vp - 1.675f * vm;
}

// WENO-Z values at Gauss point g of two row sets (the left and right
// non-equilibrium rows) with one division.  The denominators are sums of
// products of three (beta + eps) factors, eps = 1e-6, so their product stays
// far inside the double range for any bounded data.
template <typename T>
GKS_HD void tan_weno_pair(const T* ql, const T* qr, int g, T& vl, T& vr)
{
    T nl, dl, nr, dr;
    tan_weno_frac<T>(ql, g, nl, dl);
    tan_weno_frac<T>(qr, g, nr, dr);
    const T r = rcp(dl * dr);
    vl = nl * dr * r;
    vr = nr * dl * r;
}

// erfc(z) from q = exp(-z^2), which the half-range moments form anyway.
// For a = |z|: erfc(a) = q p(t) / (1 + 2a), t = (a - K) / (a + K) in
// [-1, 1), where p is a polynomial fitted to (1 + 2a) exp(a^2) erfc(a), a
// function analytic in t (the mapping of J. L. Schonfelder, Math. Comp. 32,
// 1978); then erfc(-a) = 2 - erfc(a).  One reciprocal and no branch, where
// the library's erfc picks among argument ranges (lanes of a wave in
// different ranges run several of them).  The even and odd parts of p are
// two interleaved Horner chains in t^2.  Coefficients and their error (at
// most 2.9 ulp of exp(a^2) erfc(a) over [0, 30] in either precision) from
// erfc_fit.py; other types (the operation counter) call the library.
constexpr double kErfcK64 = 3.0;
constexpr double kErfcP64[25] = {
    1.2530080582697296,     -0.13562110612458117,   -0.04756229435345087,   0.1296451587027606,
    -0.11927366341530699,   0.06830802734397848,    -0.023770514918645888,  0.002529391816066239,
    0.0018886903591561553,  -0.0007798322721083991, -0.00010515979981501177, 0.00012509935235563107,
    4.949484992570595e-06,  -2.0100567931289227e-05, -7.315105164159062e-07, 3.472414602875686e-06,
    3.5683839153992204e-07, -6.166496077604353e-07, -1.4160064940265987e-07, 1.0187000600072885e-07,
    4.180784698845582e-08,  -1.3326364813003834e-08, -8.500397929772615e-09, 9.885798831139365e-10,
    8.864219016427092e-10};
constexpr float kErfcK32 = 2.0f;
constexpr float kErfcP32[11] = {
    1.2769783735275269f,   -0.0927630364894867f,    -0.16603060066699982f, 0.16403527557849884f,
    -0.05421590059995651f, -0.007940706796944141f,  0.008700217120349407f, 0.0010404807981103659f,
    -0.0014083577552810311f, -0.00018247801926918328f, 0.00016586757556069642f};

template <typename T, int N>
GKS_HD T erfc_mapped(T z, T q, const T (&c)[N], T K)
{
    const T a = tabs(z);
    const T b = fmadd(T(2), a, T(1));
    const T r = rcp((a + K) * b);
    const T t = (a - K) * b * r;
    const T w = (a + K) * r; // 1 / (1 + 2a)
    const T t2 = t * t;
    constexpr int je = (N - 1) & ~1, jo = ((N - 2) & ~1) + 1;
    T ev = c[je], od = c[jo];
#pragma unroll
    for (int j = je - 2; j >= 0; j -= 2) ev = fmadd(ev, t2, c[j]);
#pragma unroll
    for (int j = jo - 2; j >= 1; j -= 2) od = fmadd(od, t2, c[j]);
    const T v = q * (fmadd(od, t, ev) * w);
    return z < T(0) ? T(2) - v : v;
}
template <typename T> GKS_HD T erfc_q(T z, T) { return erfc(z); }
template <> GKS_HD double erfc_q<double>(double z, double q) { return erfc_mapped(z, q, kErfcP64, kErfcK64); }
template <> GKS_HD float erfc_q<float>(float z, float q) { return erfc_mapped(z, q, kErfcP32, kErfcK32); }

// ---------------------------------------------------------------------------
// Maxwellian moments (Sec. 2.1).  For g = rho (lam/pi)^{(K+D)/2}
// exp(-lam((u-U)^2 + (v-V)^2 + xi^2)) with unit density:
//   mu[n] = <u^n> (full range, u > 0 or u < 0), mv[n] = <v^n>,
//   mx[k] = <(xi^2)^k>.  D = DIM; K internal degrees of freedom.
// ---------------------------------------------------------------------------
template <typename T, int DIM, int NU>
struct Moments {
    T U, V, lam;
    T mu[NU];
    T mv[(DIM == 2) ? 9 : 1];
    T mx[4];
};

// half: 0 full, +1 u > 0, -1 u < 0
template <typename T, int DIM, int NU>
GKS_HD void make_moments(T U, T V, T lam, T h, T K, int half, Moments<T, DIM, NU>& m)
{
    // h = 1 / (2 lam), passed in (the caller has it without a division)
    m.U = U; m.V = V; m.lam = lam;
    if (half == 0) {
        m.mu[0] = T(1);
        m.mu[1] = U;
    } else {
        const T sl = sqrt(lam);
        const T q = exp(-lam * U * U);
        // (1/2) / sqrt(pi lam) = h sqrt(lam) / sqrt(pi)
        const T e = q * (h * sl) * T(0.56418958354775628695);
        // u > 0 (half = +1) or u < 0 (half = -1), without a branch: the two
        // states of a lane pair run the same instructions
        const T s = half > 0 ? T(1) : T(-1);
        m.mu[0] = T(0.5) * erfc_q(-s * sl * U, q);
        m.mu[1] = fmadd(U, m.mu[0], s * e);
    }
#pragma unroll
    for (int n = 2; n < NU; ++n) m.mu[n] = U * m.mu[n - 1] + T(n - 1) * h * m.mu[n - 2];
    if constexpr (DIM == 2) {
        m.mv[0] = T(1);
        m.mv[1] = V;
#pragma unroll
        for (int n = 2; n < 9; ++n) m.mv[n] = V * m.mv[n - 1] + T(n - 1) * h * m.mv[n - 2];
    } else {
        m.mv[0] = T(1);
    }
    m.mx[0] = T(1);
    m.mx[1] = K * h;
    m.mx[2] = m.mx[1] * (K + T(2)) * h;
    m.mx[3] = m.mx[2] * (K + T(4)) * h;
}

// <u^A v^B Q^C>, Q = u^2 + v^2 + xi^2 (v absent in 1-D)
template <int A, int B, int C, typename M>
GKS_HD auto mom(const M& m) -> typename std::remove_reference<decltype(m.U)>::type
{
    using T = typename std::remove_reference<decltype(m.U)>::type;
    constexpr bool two = (sizeof(m.mv) / sizeof(m.mv[0])) > 1;
    if constexpr (!two) {
        static_assert(B == 0, "no v moments in 1-D");
        if constexpr (C == 0) return m.mu[A];
        else if constexpr (C == 1) return m.mu[A + 2] + m.mu[A] * m.mx[1];
        else if constexpr (C == 2) return m.mu[A + 4] + T(2) * m.mu[A + 2] * m.mx[1] + m.mu[A] * m.mx[2];
        else return m.mu[A + 6] + T(3) * m.mu[A + 4] * m.mx[1] + T(3) * m.mu[A + 2] * m.mx[2] + m.mu[A] * m.mx[3];
    } else {
        const T* u = m.mu;
        const T* v = m.mv;
        const T* x = m.mx;
        if constexpr (C == 0) return u[A] * v[B];
        else if constexpr (C == 1) return u[A + 2] * v[B] + u[A] * (v[B + 2] + v[B] * x[1]);
        else if constexpr (C == 2)
            return u[A + 4] * v[B] + u[A] * (v[B + 4] + v[B] * x[2] + T(2) * v[B + 2] * x[1]) +
                   T(2) * u[A + 2] * (v[B + 2] + v[B] * x[1]);
        else
            return u[A + 6] * v[B] + u[A] * (v[B + 6] + v[B] * x[3] + T(3) * v[B + 4] * x[1] + T(3) * v[B + 2] * x[2]) +
                   T(3) * u[A + 4] * (v[B + 2] + v[B] * x[1]) +
                   u[A + 2] * (T(3) * v[B + 4] + T(3) * v[B] * x[2] + T(6) * v[B + 2] * x[1]);
    }
}

// psi = (1, u, v, Q/2): slot -> (u power, v power, Q power)
constexpr int kPu[4] = {0, 1, 0, 0};
constexpr int kPv[4] = {0, 0, 1, 0};
constexpr int kPq[4] = {0, 0, 0, 1};

// <u^A v^B psi_K psi_P>
template <int A, int B, int K, int P, typename M>
GKS_HD auto s_elem(const M& m)
{
    using T = typename std::remove_reference<decltype(m.U)>::type;
    constexpr int c = kPq[K] + kPq[P];
    constexpr double sc = c == 0 ? 1.0 : (c == 1 ? 0.5 : 0.25);
    return T(sc) * mom<A + kPu[K] + kPu[P], B + kPv[K] + kPv[P], c>(m);
}
// <u^A v^B psi_K psi_P psi_Q>
template <int A, int B, int K, int P, int Q, typename M>
GKS_HD auto t_elem(const M& m)
{
    using T = typename std::remove_reference<decltype(m.U)>::type;
    constexpr int c = kPq[K] + kPq[P] + kPq[Q];
    constexpr double sc = c == 0 ? 1.0 : (c == 1 ? 0.5 : (c == 2 ? 0.25 : 0.125));
    return T(sc) * mom<A + kPu[K] + kPu[P] + kPu[Q], B + kPv[K] + kPv[P] + kPv[Q], c>(m);
}

template <int DIM> struct Slots;
template <> struct Slots<1> { using seq = std::integer_sequence<int, 0, 1, 3>; };
template <> struct Slots<2> { using seq = std::integer_sequence<int, 0, 1, 2, 3>; };

// out_K = sum_P a_P <u^A v^B psi_P psi_K>  (a linear in psi)
template <int A, int B, int K, typename M, typename T, int... P>
GKS_HD T lin_row(const M& m, const T* a, std::integer_sequence<int, P...>)
{
    return ((a[P] * s_elem<A, B, K, P>(m)) + ...);
}
template <int A, int B, int DIM, typename M, typename T, int... K>
GKS_HD void lin_impl(const M& m, const T* a, T* out, std::integer_sequence<int, K...>)
{
    ((out[K] = lin_row<A, B, K>(m, a, typename Slots<DIM>::seq{})), ...);
}
template <int A, int B, int DIM, typename M, typename T>
GKS_HD void lin(const M& m, const T* a, T* out)
{
    lin_impl<A, B, DIM>(m, a, out, typename Slots<DIM>::seq{});
}

// out_K = <u^A v^B psi_K>
template <int A, int B, int DIM, typename M, typename T, int... K>
GKS_HD void psi_impl(const M& m, T* out, std::integer_sequence<int, K...>)
{
    ((out[K] = s_elem<A, B, K, 0>(m)), ...);
}
template <int A, int B, int DIM, typename M, typename T>
GKS_HD void psi_mom(const M& m, T* out)
{
    psi_impl<A, B, DIM>(m, out, typename Slots<DIM>::seq{});
}

// out_K = sum_{P,Q} a_P b_Q <u^A v^B psi_P psi_Q psi_K>
template <int A, int B, int K, int P, typename M, typename T, int... Q>
GKS_HD T bil_inner(const M& m, const T* b, std::integer_sequence<int, Q...>)
{
    return ((b[Q] * t_elem<A, B, K, P, Q>(m)) + ...);
}
template <int A, int B, int K, int DIM, typename M, typename T, int... P>
GKS_HD T bil_row(const M& m, const T* a, const T* b, std::integer_sequence<int, P...>)
{
    return ((a[P] * bil_inner<A, B, K, P>(m, b, typename Slots<DIM>::seq{})) + ...);
}
template <int A, int B, int DIM, typename M, typename T, int... K>
GKS_HD void bil_impl(const M& m, const T* a, const T* b, T* out, std::integer_sequence<int, K...>)
{
    ((out[K] = bil_row<A, B, K, DIM>(m, a, b, typename Slots<DIM>::seq{})), ...);
}
template <int A, int B, int DIM, typename M, typename T>
GKS_HD void bil(const M& m, const T* a, const T* b, T* out)
{
    bil_impl<A, B, DIM>(m, a, b, out, typename Slots<DIM>::seq{});
}

// Micro-coefficients a (linear in psi) with <a psi> = b for the Maxwellian
// (U, V, lam) with unit density: the closed-form inverse of the moment
// matrix (textbook gas-kinetic solve).  K: internal degrees of freedom.
template <typename T, int DIM>
GKS_HD void micro_solve(T U, T V, T lam, T h, T N, T iN, const T* b, T* a)
{
    // h = 1 / (2 lam), N = K + DIM, iN = 1 / N
    if constexpr (DIM == 2) {
        const T e = U * U + V * V + N * h;
        const T R4 = T(2) * b[3] - e * b[0];
        const T R3 = b[2] - V * b[0];
        const T R2 = b[1] - U * b[0];
        a[3] = T(4) * iN * lam * lam * (R4 - T(2) * U * R2 - T(2) * V * R3);
        a[2] = T(2) * lam * R3 - V * a[3];
        a[1] = T(2) * lam * R2 - U * a[3];
        a[0] = b[0] - U * a[1] - V * a[2] - T(0.5) * a[3] * e;
    } else {
        const T e = U * U + N * h;
        const T R3 = T(2) * b[3] - e * b[0];
        const T R2 = b[1] - U * b[0];
        a[3] = T(4) * iN * lam * lam * (R3 - T(2) * U * R2);
        a[1] = T(2) * lam * R2 - U * a[3];
        a[2] = T(0);
        a[0] = b[0] - U * a[1] - T(0.5) * a[3] * e;
    }
}

// primitive variables of a conservative state; false if not physical
template <typename T, int DIM>
GKS_HD bool primitive(const T* W, T gamma, T& rho, T& U, T& V, T& lam, T& p, T& ir, T& ip)
{
    // ir = 1 / rho and ip = 1 / p are returned for reuse
    rho = W[0];
    ir = rcp(rho);
    U = W[1] * ir;
    V = (DIM == 2) ? W[2] * ir : T(0);
    p = (gamma - T(1)) * (W[3] - T(0.5) * rho * (U * U + V * V));
    ip = rcp(p);
    lam = T(0.5) * rho * ip;
    return (rho > T(0)) && (p > T(0));
}

template <typename T> GKS_HD bool physical(const T* W, T gamma, int dim)
{
    const T rho = W[0], ir = rcp(rho);
    const T U = W[1] * ir, V = dim == 2 ? W[2] * ir : T(0);
    const T p = (gamma - T(1)) * (W[3] - T(0.5) * rho * (U * U + V * V));
    return (rho > T(0)) && (p > T(0));
}

// ---------------------------------------------------------------------------
// Time-fit coefficients of the e^{-t/tau_n} part (reading: its time
// integrals over [0, dt/2] and [0, dt] are matched by a + b t), FP64.
// ke, kte: value coefficients of the e and t*e parts; kde, kdte: slopes.
// ---------------------------------------------------------------------------
// e^{-x} and 1 - e^{-x} for x >= 0.  In FP64 one library call: the smaller
// of the two (at most 1/2, x > ln 2 or not) is evaluated and the other is 1
// minus it, which rounds once (half an ulp).  Other types (the operation
// counter) evaluate both.
template <typename D> GKS_HD void exp_pair(D x, D& q, D& om)
{
    q = exp(-x);
    om = -expm1(-x);
}
template <> GKS_HD void exp_pair<double>(double x, double& q, double& om)
{
    if (x > 0.69314718055994531) {
        q = exp(-x);
        om = 1.0 - q;
    } else {
        om = -expm1(-x);
        q = 1.0 - om;
    }
}

template <typename D>
GKS_HD void exp_fit(D tau_n, D dt, D idt, D& ke, D& kte, D& kde, D& kdte)
{
    const D x2 = dt * rcp(tau_n), x1 = D(0.5) * x2;
    // e^{-x2} = (e^{-x1})^2 and 1 - e^{-x2} = (1 - e^{-x1})(1 + e^{-x1})
    D q1, om1; // e^{-x1}, 1 - e^{-x1}
    exp_pair(x1, q1, om1);
    const D q2 = q1 * q1, om2 = om1 * (D(1) + q1);
    const D Ie1 = tau_n * om1, Ie2 = tau_n * om2;
    const D It1 = tau_n * tau_n * om1 - tau_n * (D(0.5) * dt) * q1;
    const D It2 = tau_n * tau_n * om2 - tau_n * dt * q2;
    ke = (D(4) * Ie1 - Ie2) * idt;
    kde = D(4) * (Ie2 - D(2) * Ie1) * idt * idt;
    kte = (D(4) * It1 - It2) * idt;
    kdte = D(4) * (It2 - D(2) * It1) * idt * idt;
}

// ---------------------------------------------------------------------------
// Central-velocity form of the equilibrium moments.  With c = u - U,
// w = v - V and phi = (1, c, w, Q/2), Q = c^2 + w^2 + xi^2, the Maxwellian's
// moments are closed forms in h = 1/(2 lambda) and N = K + D (isotropic
// Gaussian with variance h per degree of freedom):
//   <c^a w^b Q^k> = 0 for odd a or b, else
//   h^{a/2+b/2+k} (a-1)!! (b-1)!! prod_{m<k} (N + a + b + 2m).
// psi = M phi with M lower triangular (psi_1 = U + c, psi_2 = V + w,
// psi_3 = E0 + U c + V w + phi_3, E0 = (U^2 + V^2)/2), so moment conditions
// <(a.psi) psi> = b become G a^ = M^{-1} b with a^ = M^T a and the almost
// diagonal Gram matrix G = <phi phi^T>.
// ---------------------------------------------------------------------------
template <typename T>
struct Central {
    T h[7]; // h^n
    T N;
    T U, V, E0;
    T ih, iN; // 1/h, 1/N (shared by every Gram solve of the point)
};

constexpr double dfact(int n) { return n <= 0 ? 1.0 : double(n) * dfact(n - 2); }
constexpr int kCc[4] = {0, 1, 0, 0};
constexpr int kCw[4] = {0, 0, 1, 0};
constexpr int kCq[4] = {0, 0, 0, 1};

template <int A, int B> constexpr bool odd_cw() { return (A % 2) != 0 || (B % 2) != 0; }

// <c^A w^B Q^Kq>, A and B even
template <int A, int B, int Kq, typename T>
GKS_HD T mc(const Central<T>& C)
{
    static_assert(!odd_cw<A, B>(), "odd central moments vanish");
    constexpr int e = A / 2 + B / 2 + Kq;
    constexpr double df = dfact(A - 1) * dfact(B - 1);
    T v = T(df) * C.h[e];
    if constexpr (Kq >= 1) v *= C.N + T(A + B);
    if constexpr (Kq >= 2) v *= C.N + T(A + B + 2);
    if constexpr (Kq >= 3) v *= C.N + T(A + B + 4);
    return v;
}

// 2-tensor <c^Al w^Be phi_J phi_P> and 3-tensor <c^Al w^Be phi_J phi_P phi_R>
template <int Al, int Be, int J, int P> constexpr bool z2() { return odd_cw<Al + kCc[J] + kCc[P], Be + kCw[J] + kCw[P]>(); }
template <int Al, int Be, int J, int P, int R> constexpr bool z3()
{
    return odd_cw<Al + kCc[J] + kCc[P] + kCc[R], Be + kCw[J] + kCw[P] + kCw[R]>();
}
template <int Al, int Be, int J, int P, typename T>
GKS_HD T c2(const Central<T>& C)
{
    constexpr int q = kCq[J] + kCq[P];
    constexpr double sc = q == 0 ? 1.0 : (q == 1 ? 0.5 : 0.25);
    return T(sc) * mc<Al + kCc[J] + kCc[P], Be + kCw[J] + kCw[P], q>(C);
}
template <int Al, int Be, int J, int P, int R, typename T>
GKS_HD T c3(const Central<T>& C)
{
    constexpr int q = kCq[J] + kCq[P] + kCq[R];
    constexpr double sc = q == 0 ? 1.0 : (q == 1 ? 0.5 : (q == 2 ? 0.25 : 0.125));
    return T(sc) * mc<Al + kCc[J] + kCc[P] + kCc[R], Be + kCw[J] + kCw[P] + kCw[R], q>(C);
}

template <int Al, int Be, int J, int P, typename T>
GKS_HD void c2_acc(const Central<T>& C, const T* a, T& acc)
{
    if constexpr (!z2<Al, Be, J, P>()) acc += a[P] * c2<Al, Be, J, P>(C);
}
template <int Al, int Be, int J, int P, int R, typename T>
GKS_HD void c3_acc(const Central<T>& C, const T* a, const T* b, T& acc)
{
    if constexpr (!z3<Al, Be, J, P, R>()) acc += (a[P] * b[R]) * c3<Al, Be, J, P, R>(C);
}
template <int Al, int Be, int J, typename T, int... P>
GKS_HD T c2_row(const Central<T>& C, const T* a, std::integer_sequence<int, P...>)
{
    T acc = T(0);
    (c2_acc<Al, Be, J, P>(C, a, acc), ...);
    return acc;
}
template <int Al, int Be, int J, int P, typename T, int... R>
GKS_HD void c3_inner(const Central<T>& C, const T* a, const T* b, T& acc, std::integer_sequence<int, R...>)
{
    (c3_acc<Al, Be, J, P, R>(C, a, b, acc), ...);
}
template <int Al, int Be, int J, int DIM, typename T, int... P>
GKS_HD T c3_row(const Central<T>& C, const T* a, const T* b, std::integer_sequence<int, P...>)
{
    T acc = T(0);
    (c3_inner<Al, Be, J, P>(C, a, b, acc, typename Slots<DIM>::seq{}), ...);
    return acc;
}
template <int Al, int Be, int DIM, typename T, int... J>
GKS_HD void clin_impl(const Central<T>& C, const T* a, T* out, std::integer_sequence<int, J...>)
{
    ((out[J] = c2_row<Al, Be, J>(C, a, typename Slots<DIM>::seq{})), ...);
}
template <int Al, int Be, int DIM, typename T, int... J>
GKS_HD void cbil_impl(const Central<T>& C, const T* a, const T* b, T* out, std::integer_sequence<int, J...>)
{
    ((out[J] = c3_row<Al, Be, J, DIM>(C, a, b, typename Slots<DIM>::seq{})), ...);
}
// out_J = <c^Al w^Be (a.phi) phi_J>
template <int Al, int Be, int DIM, typename T>
GKS_HD void clin(const Central<T>& C, const T* a, T* out)
{
    clin_impl<Al, Be, DIM>(C, a, out, typename Slots<DIM>::seq{});
}
// out_J = <c^Al w^Be (a.phi)(b.phi) phi_J>
template <int Al, int Be, int DIM, typename T>
GKS_HD void cbil(const Central<T>& C, const T* a, const T* b, T* out)
{
    cbil_impl<Al, Be, DIM>(C, a, b, out, typename Slots<DIM>::seq{});
}

// b^ = M^{-1} b (conservative-variable vector -> central dual basis)
template <typename T, int DIM>
GKS_HD void to_central(const Central<T>& C, const T* b, T s, T* o)
{
    o[0] = s * b[0];
    o[1] = s * (b[1] - C.U * b[0]);
    o[2] = DIM == 2 ? s * (b[2] - C.V * b[0]) : T(0);
    o[3] = s * (b[3] - C.U * b[1] - (DIM == 2 ? C.V * b[2] : T(0)) + C.E0 * b[0]);
}
// b = M b^ (central dual -> conservative-variable vector), scaled by s
template <typename T, int DIM>
GKS_HD void from_central(const Central<T>& C, const T* o, T s, T* b)
{
    b[0] = s * o[0];
    b[1] = s * (C.U * o[0] + o[1]);
    b[2] = DIM == 2 ? s * (C.V * o[0] + o[2]) : T(0);
    b[3] = s * (C.E0 * o[0] + C.U * o[1] + (DIM == 2 ? C.V * o[2] : T(0)) + o[3]);
}
// a^ = G^{-1} b^
template <typename T, int DIM>
GKS_HD void gsolve(const Central<T>& C, const T* b, T* a)
{
    const T ih = C.ih;
    a[1] = b[1] * ih;
    a[2] = DIM == 2 ? b[2] * ih : T(0);
    a[0] = T(0.5) * (C.N + T(2)) * b[0] - b[3] * ih;
    a[3] = -b[0] * ih + T(2) * b[3] * ih * ih * C.iN;
}

// ---------------------------------------------------------------------------
// The interface point: simplified third-order distribution (Sec. 2.1)
//   f = g0 [1 + Abar t + G_tt t^2/2] - tau g0 [(abar.u + Abar) + (G_xt u + G_yt v + G_tt) t]
//       + e^{-t/tau_n} { -g0 [1 - abar.u t] + g_l [1 - a_l.u t] H(u) + g_r [1 - a_r.u t] (1-H(u)) }
// G_.. are the exact second Taylor coefficients of the Maxwellian over g0.
// Outputs (type D, FP64): FL (flux giving L), FdL (flux giving dL/dt), S0,
// S1, S2 (moments of f^n, f_t^n, f_tt^n).  Local frame (normal = slot 1).
// Precision split: the O(1) quantities (equilibrium value, its Euler flux,
// the half-range moments of the two states) are of type D; everything
// proportional to a reconstructed derivative is of type T.
// ---------------------------------------------------------------------------
template <typename T>
struct PointIn {
    T W0x[4], W0y[4], W0xx[4], W0xy[4], W0yy[4];
    T Wlx[4], Wly[4], Wrx[4], Wry[4];
};
template <typename D>
struct PointOut {
    D FL[4], FdL[4], S0[4], S1[4], S2[4];
};

// Per-launch constants of the interface point, with the reciprocals formed
// once per launch instead of at every point: idt = 1 / dt, iN = 1 / (K + DIM).
struct PointPar {
    double gamma, K, mu, dt, idt, iN;
};
template <int DIM>
GKS_HD PointPar point_par(double gamma, double K, double mu, double dt)
{
    return PointPar{gamma, K, mu, dt, 1.0 / dt, 1.0 / (K + DIM)};
}

template <typename D, int NU, int DIM, typename T>
GKS_HD void cast_moments(const Moments<D, DIM, NU>& a, Moments<T, DIM, NU>& b)
{
    b.U = T(a.U); b.V = T(a.V); b.lam = T(a.lam);
#pragma unroll
    for (int n = 0; n < NU; ++n) b.mu[n] = T(a.mu[n]);
#pragma unroll
    for (int n = 0; n < (DIM == 2 ? 9 : 1); ++n) b.mv[n] = T(a.mv[n]);
#pragma unroll
    for (int n = 0; n < 4; ++n) b.mx[n] = T(a.mx[n]);
}

// The two non-equilibrium states at the point (Sec. 2.1, the g_l, g_r terms):
//   Xs = <psi>_{l,u>0} + <psi>_{r,u<0},  Xf = <u psi>_{l,u>0} + <u psi>_{r,u<0}
// (type D), their pressures, and (type T, only when slopes are given)
//   Hn = <(a_l.u) psi>_{l,u>0} + <(a_r.u) psi>_{r,u<0},
//   Hm = <u (a_l.u) psi>_{l,u>0} + <u (a_r.u) psi>_{r,u<0},
// with a_l, a_r the micro-slopes of the states' normal (and tangential)
// derivatives.
template <typename D, int DIM, typename T = D>
struct NonEq {
    D pl, pr;
    D Xs[4], Xf[4];
    T Hn[4], Hm[4];
};

// One state's share: its pressure and density and, per unit density, its
// half-range moments h0 = <psi>, h1 = <u psi> (type D) and, when slopes are
// given, h2 = <(a.u) psi>, h3 = <u (a.u) psi> (type T).  side 0: the left
// state over u > 0; side 1: the right state over u < 0.
template <typename D, int DIM, typename T = D>
struct NeSide {
    D p, rs;
    D h0[4], h1[4];
    T rt;
    T h2[4], h3[4];
};

template <typename D, int DIM, typename T = D>
GKS_HD bool noneq_side(const D* Ws, int side, D gamma, D K, D iN, NeSide<D, DIM, T>& o, const T* Wn = nullptr,
                       const T* Wt = nullptr)
{
    D rs, Us, Vs, ls, ps, irs_d, ips;
    const bool ok = primitive<D, DIM>(Ws, gamma, rs, Us, Vs, ls, ps, irs_d, ips);
    const D hs = ps * irs_d; // 1 / (2 lam) = p / rho
    o.p = ps;
    o.rs = rs;
    Moments<D, DIM, 7> m;
    make_moments<D, DIM, 7>(Us, Vs, ls, hs, K, side ? -1 : +1, m);
    psi_mom<0, 0, DIM>(m, o.h0);
    psi_mom<1, 0, DIM>(m, o.h1);
    o.rt = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) { o.h2[k] = T(0); o.h3[k] = T(0); }
    if (Wn) {
        Moments<T, DIM, 7> mt;
        cast_moments<D, 7, DIM, T>(m, mt);
        const T irs = T(irs_d), h_t = T(hs), N_t = T(K) + T(DIM), iN_t = T(iN);
        o.rt = T(rs);
        T b[4], as1[4], as2[4] = {T(0), T(0), T(0), T(0)}, t1[4], t2[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) b[k] = Wn[k] * irs;
        micro_solve<T, DIM>(mt.U, mt.V, mt.lam, h_t, N_t, iN_t, b, as1);
        if constexpr (DIM == 2) {
#pragma unroll
            for (int k = 0; k < 4; ++k) b[k] = Wt[k] * irs;
            micro_solve<T, DIM>(mt.U, mt.V, mt.lam, h_t, N_t, iN_t, b, as2);
        }
        lin<1, 0, DIM>(mt, as1, o.h2); // <a1 u psi>_half
        lin<2, 0, DIM>(mt, as1, o.h3); // <a1 u^2 psi>_half
        if constexpr (DIM == 2) {
            lin<0, 1, DIM>(mt, as2, t1);
            lin<1, 1, DIM>(mt, as2, t2);
#pragma unroll
            for (int k = 0; k < 4; ++k) { o.h2[k] += t1[k]; o.h3[k] += t2[k]; }
        }
    }
    return ok;
}

// The two states' sums, left share first: X = rs_r h_r + rs_l h_l (fused).
template <typename D, int DIM, typename T = D>
GKS_HD void noneq_combine(const NeSide<D, DIM, T>& l, const NeSide<D, DIM, T>& r, NonEq<D, DIM, T>& ne)
{
    ne.pl = l.p;
    ne.pr = r.p;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ne.Xs[k] = fmadd(r.rs, r.h0[k], l.rs * l.h0[k]);
        ne.Xf[k] = fmadd(r.rs, r.h1[k], l.rs * l.h1[k]);
        ne.Hn[k] = fmadd(r.rt, r.h2[k], l.rt * l.h2[k]);
        ne.Hm[k] = fmadd(r.rt, r.h3[k], l.rt * l.h3[k]);
    }
}

template <typename D, int DIM, typename T = D>
GKS_HD bool noneq_states(const D* Wl, const D* Wr, D gamma, D K, D iN, NonEq<D, DIM, T>& ne, const T* Wlx = nullptr,
                         const T* Wly = nullptr, const T* Wrx = nullptr, const T* Wry = nullptr)
{
    NeSide<D, DIM, T> l, r;
    if (!noneq_side<D, DIM, T>(Wl, 0, gamma, K, iN, l, Wlx, Wly)) return false;
    if (!noneq_side<D, DIM, T>(Wr, 1, gamma, K, iN, r, Wrx, Wry)) return false;
    noneq_combine<D, DIM, T>(l, r, ne);
    return true;
}

// W0d: equilibrium state (type D); ne: the two non-equilibrium states.
// Returns false for a non-physical equilibrium state.
template <typename T, int DIM, typename D = double>
GKS_HD bool gks_point(const PointPar& par, const PointIn<T>& in, const D* W0d, const NonEq<D, DIM, T>& ne,
                      PointOut<D>& out)
{
    const D gammad = D(par.gamma);
    D r0d, U0d, V0d, l0d, p0d, ir0d, ip0d;
    if (!primitive<D, DIM>(W0d, gammad, r0d, U0d, V0d, l0d, p0d, ir0d, ip0d)) return false;

    // collision times (Sec. 4): the Navier-Stokes terms take mu/p (0 for
    // Euler) plus the pressure-jump term, the artificial dissipation of
    // discontinuities; the exponentials take the full tau_n (epsilon dt for
    // Euler, mu/p for Navier-Stokes, plus the jump term)
    const D dtd = D(par.dt);
    const D jump = tabs(quot(ne.pl - ne.pr, ne.pl + ne.pr)) * dtd;
    const D tau_d = (par.mu > 0.0 ? D(par.mu) * ip0d : D(0)) + jump;
    const D tau_n = par.mu > 0.0 ? tau_d : D(0.01) * dtd + jump;
    D ke, kte, kde, kdte;
    {
        using E = ExpT<D>;
        E ke_, kte_, kde_, kdte_;
        exp_fit<E>(E(tau_n), E(par.dt), E(par.idt), ke_, kte_, kde_, kdte_);
        ke = D(ke_); kte = D(kte_); kde = D(kde_); kdte = D(kdte_);
    }

    // ---- equilibrium part in central velocities (type T) ----
    Central<T> C;
    const T r0 = T(r0d), ir0 = T(ir0d);
    C.U = T(U0d);
    C.V = T(V0d);
    C.E0 = T(0.5) * (C.U * C.U + C.V * C.V);
    C.N = T(par.K) + T(DIM);
    C.h[0] = T(1);
    C.h[1] = T(p0d * ir0d);
    C.ih = T(r0d * ip0d);
    C.iN = T(par.iN);
#pragma unroll
    for (int n = 2; n < 7; ++n) C.h[n] = C.h[n - 1] * C.h[1];
    const T U = C.U, V = C.V;
    const T tau = T(tau_d);

    // The outputs are sums of separately formed terms:
    //   FL  = F0 - tau <u(a.u + Abar)psi> + ke Me + kte Mte
    //   FdL = <u Abar psi> - tau <u(G_xt u + G_yt v + G_tt)psi> + kde Me + kdte Mte
    //   S0  = W0 + ke Ne + kte Nte,  S1 = <Abar psi> + kde Ne + kdte Nte,  S2 = <G_tt psi>
    // with Me = Xf - F0, Ne = Xs - W0 (values of the two states) and
    // Mte = <u(a.u)psi>_0 - Hm, Nte = -<Abar psi> - Hn (their slope parts).
    // Each term is added as soon as it is formed, so the intermediate
    // vectors do not stay live to the end.
    {
        D F0[4];
        F0[0] = W0d[1];
        F0[1] = W0d[1] * U0d + p0d;
        F0[2] = W0d[2] * U0d;
        F0[3] = U0d * (W0d[3] + p0d);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const D Me = ne.Xf[k] - F0[k];
            const D Ne = ne.Xs[k] - W0d[k];
            const D hm = D(ne.Hm[k]), hn = D(ne.Hn[k]);
            out.FL[k] = F0[k] + ke * Me - kte * hm;
            out.FdL[k] = kde * Me - kdte * hm;
            out.S0[k] = W0d[k] + ke * Ne - kte * hn;
            out.S1[k] = kde * Ne - kdte * hn;
        }
    }
    T a1[4], a2[4] = {T(0), T(0), T(0), T(0)}, At[4], t1[4], t2[4];
    {
        T bx[4], by[4] = {T(0), T(0), T(0), T(0)};
        to_central<T, DIM>(C, in.W0x, ir0, bx);
        if constexpr (DIM == 2) to_central<T, DIM>(C, in.W0y, ir0, by);
        gsolve<T, DIM>(C, bx, a1);
        if constexpr (DIM == 2) gsolve<T, DIM>(C, by, a2);
        // <u (a1 u + a2 v) psi>0 (initial-layer slope term of g0), central form
        T Mc[4];
        clin<1, 0, DIM>(C, a1, t1);
        clin<2, 0, DIM>(C, a1, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) Mc[k] = U * U * bx[k] + T(2) * U * t1[k] + t2[k];
        // compatibility: G Abar = -(U b_x + <c a1 phi> + V b_y + <w a2 phi>)
        T S1c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) S1c[k] = -(U * bx[k] + t1[k]);
        if constexpr (DIM == 2) {
            T t3[4];
            clin<0, 1, DIM>(C, a2, t3);
            clin<1, 0, DIM>(C, a2, t1);
            clin<1, 1, DIM>(C, a2, t2);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                Mc[k] += U * V * by[k] + U * t3[k] + V * t1[k] + t2[k];
                S1c[k] -= V * by[k] + t3[k];
            }
        }
        gsolve<T, DIM>(C, S1c, At);
        // <u Abar psi> = central U <Abar phi> + <c Abar phi>
        T F1c[4];
        clin<1, 0, DIM>(C, At, t1);
#pragma unroll
        for (int k = 0; k < 4; ++k) F1c[k] = U * S1c[k] + t1[k];
        T Mte[4], F1[4], S1n[4];
        from_central<T, DIM>(C, Mc, r0, Mte);
        from_central<T, DIM>(C, F1c, r0, F1);
        from_central<T, DIM>(C, S1c, r0, S1n);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            out.FL[k] += kte * D(Mte[k]);
            out.FdL[k] += D(F1[k]) + kdte * D(Mte[k]);
            out.S0[k] -= kte * D(S1n[k]);
            out.S1[k] += D(S1n[k]) - kdte * D(S1n[k]);
        }
        // Navier-Stokes: <u (a1 u + a2 v + Abar) psi> = Mc + F1c
        if (tau_d != D(0))
#pragma unroll
            for (int k = 0; k < 4; ++k) out.FL[k] -= D(tau * (Mte[k] + F1[k]));
    }
    // second-order coefficients: <G_xx phi> = b_xx etc.;
    // <G_xt phi> = -<(U + c) G_xx phi> - <(V + w) G_xy phi>  (= Pxt), same for yt
    T Pxt[4], Pyt[4] = {T(0), T(0), T(0), T(0)};
    {
        T bxx[4], axx[4];
        to_central<T, DIM>(C, in.W0xx, ir0, bxx);
        cbil<0, 0, DIM>(C, a1, a1, t1);
#pragma unroll
        for (int k = 0; k < 4; ++k) t1[k] = bxx[k] - t1[k];
        gsolve<T, DIM>(C, t1, axx);
        clin<1, 0, DIM>(C, axx, t1);
        cbil<1, 0, DIM>(C, a1, a1, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) Pxt[k] = -(U * bxx[k] + t1[k] + t2[k]);
    }
    if constexpr (DIM == 2) {
        T bxy[4], axy[4];
        to_central<T, DIM>(C, in.W0xy, ir0, bxy);
        cbil<0, 0, DIM>(C, a1, a2, t1);
#pragma unroll
        for (int k = 0; k < 4; ++k) t1[k] = bxy[k] - t1[k];
        gsolve<T, DIM>(C, t1, axy);
        clin<0, 1, DIM>(C, axy, t1);
        cbil<0, 1, DIM>(C, a1, a2, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) Pxt[k] -= V * bxy[k] + t1[k] + t2[k];
        clin<1, 0, DIM>(C, axy, t1);
        cbil<1, 0, DIM>(C, a1, a2, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) Pyt[k] = -(U * bxy[k] + t1[k] + t2[k]);
        T byy[4], ayy[4];
        to_central<T, DIM>(C, in.W0yy, ir0, byy);
        cbil<0, 0, DIM>(C, a2, a2, t1);
#pragma unroll
        for (int k = 0; k < 4; ++k) t1[k] = byy[k] - t1[k];
        gsolve<T, DIM>(C, t1, ayy);
        clin<0, 1, DIM>(C, ayy, t1);
        cbil<0, 1, DIM>(C, a2, a2, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) Pyt[k] -= V * byy[k] + t1[k] + t2[k];
    }
    T axt[4], ayt[4] = {T(0), T(0), T(0), T(0)};
    cbil<0, 0, DIM>(C, a1, At, t1);
#pragma unroll
    for (int k = 0; k < 4; ++k) t1[k] = Pxt[k] - t1[k];
    gsolve<T, DIM>(C, t1, axt);
    if constexpr (DIM == 2) {
        cbil<0, 0, DIM>(C, a2, At, t1);
#pragma unroll
        for (int k = 0; k < 4; ++k) t1[k] = Pyt[k] - t1[k];
        gsolve<T, DIM>(C, t1, ayt);
    }
    // <G_tt phi> = -<(U + c) G_xt phi> - <(V + w) G_yt phi>
    T S2c[4], cx[4], cy[4] = {T(0), T(0), T(0), T(0)};
    clin<1, 0, DIM>(C, axt, t1);
    cbil<1, 0, DIM>(C, a1, At, t2);
#pragma unroll
    for (int k = 0; k < 4; ++k) { cx[k] = t1[k] + t2[k]; S2c[k] = -(U * Pxt[k] + cx[k]); } // cx = <c G_xt phi>
    if constexpr (DIM == 2) {
        clin<0, 1, DIM>(C, ayt, t1);
        cbil<0, 1, DIM>(C, a2, At, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) { cy[k] = t1[k] + t2[k]; S2c[k] -= V * Pyt[k] + cy[k]; } // cy = <w G_yt phi>
    }
    {
        T S2n[4];
        from_central<T, DIM>(C, S2c, r0, S2n);
#pragma unroll
        for (int k = 0; k < 4; ++k) out.S2[k] = D(S2n[k]);
    }
    if (tau_d != D(0)) {
        // <u (G_xt u + G_yt v + G_tt) psi>
        T F1t[4], att[4];
        cbil<0, 0, DIM>(C, At, At, t1);
#pragma unroll
        for (int k = 0; k < 4; ++k) t1[k] = S2c[k] - t1[k];
        gsolve<T, DIM>(C, t1, att);
        clin<2, 0, DIM>(C, axt, t1);
        cbil<2, 0, DIM>(C, a1, At, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) F1t[k] = U * U * Pxt[k] + T(2) * U * cx[k] + t1[k] + t2[k];
        clin<1, 0, DIM>(C, att, t1);
        cbil<1, 0, DIM>(C, At, At, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) F1t[k] += U * S2c[k] + t1[k] + t2[k];
        if constexpr (DIM == 2) {
            T t3[4];
            clin<1, 0, DIM>(C, ayt, t1);
            cbil<1, 0, DIM>(C, a2, At, t2);
            clin<1, 1, DIM>(C, ayt, t3);
#pragma unroll
            for (int k = 0; k < 4; ++k) F1t[k] += U * V * Pyt[k] + U * cy[k] + V * (t1[k] + t2[k]) + t3[k];
            cbil<1, 1, DIM>(C, a2, At, t3);
#pragma unroll
            for (int k = 0; k < 4; ++k) F1t[k] += t3[k];
        }
        from_central<T, DIM>(C, F1t, r0, t1);
#pragma unroll
        for (int k = 0; k < 4; ++k) out.FdL[k] -= D(tau * t1[k]);
    }
    if constexpr (DIM == 1) {
        out.FL[2] = out.FdL[2] = out.S0[2] = out.S1[2] = out.S2[2] = D(0);
    }
    return true;
}

} // namespace gks
