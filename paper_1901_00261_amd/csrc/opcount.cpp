// opcount.cpp -- algorithmic operation count of the interface arithmetic.
//
// Host program: instantiates the same templates the kernels use
// (face_recon, gp_inputs, kinetic_average, gks_point) with a counting scalar
// type and tallies every +, -, *, / and every sqrt / exp / expm1 / erfc they
// perform on one representative smooth input.  Sign changes and comparisons
// are not counted.  The counts are per unit of work of the kernels:
//   face_row_2d : one face row of the 2-D face-row kernel (WENO-Z mode)
//   gauss_point : one Gauss point of the 2-D interface kernel (inputs,
//                 kinetic average, interface distribution)
//   face_1d     : one face of the 1-D interface kernel
// Output: JSON on stdout.
#include "gks_kernels.h"

#include <cstdio>
#include <cstring>

namespace cnt {
long long add = 0, mul = 0, dv = 0, trans = 0;
}

struct Cnt {
    double v;
    Cnt() : v(0) {}
    Cnt(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator float() const { return (float)v; }
};
inline Cnt operator+(Cnt a, Cnt b) { ++cnt::add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++cnt::add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++cnt::mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++cnt::dv; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline Cnt sqrt(Cnt a) { ++cnt::trans; return Cnt(std::sqrt(a.v)); }
inline Cnt exp(Cnt a) { ++cnt::trans; return Cnt(std::exp(a.v)); }
inline Cnt expm1(Cnt a) { ++cnt::trans; return Cnt(std::expm1(a.v)); }
inline Cnt erfc(Cnt a) { ++cnt::trans; return Cnt(std::erfc(a.v)); }

struct Tally {
    long long add, mul, dv, trans;
};
static Tally snap() { return {cnt::add, cnt::mul, cnt::dv, cnt::trans}; }
static Tally diff(Tally a, Tally b) { return {b.add - a.add, b.mul - a.mul, b.dv - a.dv, b.trans - a.trans}; }
static void emit(const char* name, Tally t, bool comma)
{
    printf("  \"%s\": {\"add\": %lld, \"mul\": %lld, \"div\": %lld, \"trans\": %lld, \"flops\": %lld}%s\n", name, t.add,
           t.mul, t.dv, t.trans, t.add + t.mul + t.dv + t.trans, comma ? "," : "");
}

static void smooth_state(Cnt* W, double s)
{
    const double rho = 1.0 + 0.1 * s, U = 0.3 - 0.05 * s, V = -0.2 + 0.04 * s, p = 1.0 + 0.07 * s;
    W[0] = rho; W[1] = rho * U; W[2] = rho * V; W[3] = p / 0.4 + 0.5 * rho * (U * U + V * V);
}

int main()
{
    const double gamma = 1.4, K2 = (4.0 - 2.0 * gamma) / (gamma - 1.0), K1 = (3.0 - gamma) / (gamma - 1.0);
    printf("{\n");
    // ---- 2-D face row, 8th order, WENO-Z
    {
        Cnt Wk[4][4], Dk[4][4], o[7][4];
        for (int q = 0; q < 4; ++q) {
            smooth_state(Wk[q], 0.1 * q);
            for (int k = 0; k < 4; ++k) Dk[q][k] = 0.01 * (k + 1) * (q + 1);
        }
        Tally a = snap();
        gks::face_recon<Cnt, 2, 8, Cnt>(Wk, Dk, Cnt(0.01), Cnt(gamma), true, [&](int q, int k, Cnt v) { o[q][k] = v; });
        emit("face_row_2d", diff(a, snap()), true);
    }
    // ---- 2-D Gauss point (NS: mu > 0; and Euler), WENO-Z, averaged over the 3 points
    for (int ns = 1; ns >= 0; --ns) {
        Cnt rows[7][4][5];
        for (int r = 0; r < 5; ++r) {
            Cnt s[4];
            smooth_state(s, 0.05 * r);
            for (int k = 0; k < 4; ++k) {
                rows[0][k][r] = s[k]; rows[3][k][r] = s[k]; rows[4][k][r] = s[k];
                rows[1][k][r] = 0.1 * (k + 1); rows[2][k][r] = 0.01 * (k + 2);
                rows[5][k][r] = 0.1 * (k + 1); rows[6][k][r] = 0.1 * (k + 1);
            }
        }
        auto rv = [&](int q, int k, int r) { return rows[q][k][r]; };
        const gks::PointPar par{gamma, K2, ns ? 1e-4 : 0.0, 1e-3};
        Tally a = snap();
        bool ok = true;
        auto one = [&](int G) {
            gks::PointIn<Cnt> in;
            gks::PointOut<Cnt> out;
            Cnt W0[4], Wl[4], Wr[4];
            gks::gp_inputs<Cnt, Cnt>(rv, G, Cnt(0.01), true, Cnt(gamma), in, W0, Wl, Wr);
            gks::NonEq<Cnt, 2> ne;
            ok = ok && gks::noneq_states<Cnt, 2>(Wl, Wr, Cnt(gamma), Cnt(K2), ne, in.Wlx, in.Wly, in.Wrx, in.Wry) &&
                 gks::gks_point<Cnt, 2, Cnt>(par, in, ne.Xs, ne, out);
        };
        one(0);
        one(1);
        one(2);
        if (!ok) {
            fprintf(stderr, "opcount: unexpected non-physical sample\n");
            return 1;
        }
        Tally t = diff(a, snap());
        t.add /= 3; t.mul /= 3; t.dv /= 3; t.trans /= 3;
        emit(ns ? "gauss_point_ns" : "gauss_point_euler", t, true);
    }
    // ---- 1-D face, 8th order, WENO-Z, Euler
    {
        Cnt Wk[4][4], Dk[4][4], o[7][4];
        for (int q = 0; q < 4; ++q) {
            smooth_state(Wk[q], 0.1 * q);
            Wk[q][2] = 0.0;
            Wk[q][3] = 1.0 / 0.4 + 0.5 * Wk[q][1].v * Wk[q][1].v / Wk[q][0].v;
            for (int k = 0; k < 4; ++k) Dk[q][k] = k == 2 ? 0.0 : 0.01 * (k + 1) * (q + 1);
        }
        Tally a = snap();
        bool ok = gks::face_recon<Cnt, 1, 8, Cnt>(Wk, Dk, Cnt(0.01), Cnt(gamma), true, [&](int q, int k, Cnt v) { o[q][k] = v; });
        gks::PointIn<Cnt> in;
        gks::PointOut<Cnt> out;
        for (int k = 0; k < 4; ++k) {
            in.W0x[k] = o[1][k]; in.W0xx[k] = o[2][k];
            in.W0y[k] = in.W0xy[k] = in.W0yy[k] = 0.0;
            in.Wlx[k] = o[5][k]; in.Wrx[k] = o[6][k];
            in.Wly[k] = in.Wry[k] = 0.0;
        }
        gks::NonEq<Cnt, 1> ne;
        ok = ok && gks::noneq_states<Cnt, 1>(o[3], o[4], Cnt(gamma), Cnt(K1), ne, in.Wlx, in.Wly, in.Wrx, in.Wry);
        const gks::PointPar par{gamma, K1, 0.0, 1e-3};
        ok = ok && gks::gks_point<Cnt, 1, Cnt>(par, in, ne.Xs, ne, out);
        if (!ok) {
            fprintf(stderr, "opcount: unexpected non-physical sample\n");
            return 1;
        }
        emit("face_1d", diff(a, snap()), false);
    }
    printf("}\n");
    return 0;
}
