// opcount.cpp -- algorithmic operation count of the interface arithmetic.
//
// Host program: instantiates the same templates the kernels use
// (face_recon, gp_inputs, noneq_states, gks_point) with a counting scalar
// type and tallies the +, -, *, / and sqrt / exp / expm1 / erfc on which
// the unit's outputs depend, for one representative smooth input.  Sign
// changes and comparisons are not counted; a fused multiply-add counts as
// two operations.  The counts are per unit of work of the kernels:
//   face_row_2d        : one face row of the 2-D face-row kernel (WENO-Z)
//   gauss_point_*      : one Gauss point of the 2-D interface kernel
//                        (tangential inputs, kinetic average, interface
//                        distribution); *_s2: outputs of the second stage
//                        only (flux time derivative, second time
//                        derivative of the interface state)
//   face_1d, face_1d_s2: one face of the 1-D stage kernel
// Output: JSON on stdout.
#include "gks_kernels.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include <string>
#include <unordered_map>
#include <utility>

// Every arithmetic result is a node of an expression graph (operation kind
// and operands); a unit's count is the number of nodes its outputs depend
// on, so work whose result is not used by the requested outputs (for
// example the flux value in the second MSMD stage, which needs only the
// flux time derivative and the second time derivative of the interface
// state) is not counted.  The graph counts what a compiler must execute:
//   - operations on compile-time constants and launch parameters only are
//     folded (no node);
//   - multiplications and divisions by an exact +-1, multiplications by 0
//     and additions of 0 are folded;
//   - a sign change is free (an operand modifier) and is carried as a sign
//     bit, so x - y and x + (-y) are the same node;
//   - an operation identical to an earlier one (same kind, same operands up
//     to order for + and *) is the same node (common subexpressions).
namespace cnt {
enum Kind : unsigned char { ADD, MUL, DIV, TRANS };
struct Node {
    Kind k;
    int a, b;
};
std::vector<Node> g;
std::unordered_map<std::string, int> memo;
int make(Kind k, int sub, int a, bool na, int b, bool nb)
{
    char key[96];
    snprintf(key, sizeof key, "%d:%d:%d%c:%d%c", (int)k, sub, a, na ? '-' : '+', b, nb ? '-' : '+');
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    g.push_back({k, a, b});
    const int id = (int)g.size() - 1;
    memo.emplace(key, id);
    return id;
}
} // namespace cnt

// id >= 0: a node; -1: a compile-time constant or launch parameter; <= -3:
// an input datum (each its own leaf)
struct Cnt {
    double v;
    int id;
    bool neg; // the value is minus that of node id
    Cnt() : v(0), id(-1), neg(false) {}
    Cnt(double x) : v(x), id(-1), neg(false) {}
    Cnt(double x, int i, bool n = false) : v(x), id(i), neg(n) {}
    explicit operator double() const { return v; }
    explicit operator float() const { return (float)v; }
};
inline int& next_data()
{
    static int n = -3;
    return n;
}
inline Cnt data(double x) { return Cnt(x, next_data()--); }
inline bool is_const(const Cnt& a) { return a.id == -1; }
inline int key_id(const Cnt& a) { return a.id; }

inline Cnt operator-(Cnt a) { return Cnt(-a.v, a.id, a.id != -1 ? !a.neg : false); }
inline Cnt add(Cnt a, Cnt b, double v)
{
    if (is_const(a) && is_const(b)) return Cnt(v);
    if (is_const(a) && a.v == 0.0) return b;
    if (is_const(b) && b.v == 0.0) return a;
    // (-a) + (-b) = -(a + b); order the operands (commutative)
    bool flip = false;
    if (a.neg && b.neg) { a.neg = b.neg = false; flip = true; }
    if (a.id > b.id || (a.id == b.id && a.neg > b.neg)) std::swap(a, b);
    const int n = cnt::make(cnt::ADD, 0, a.id, a.neg, b.id, b.neg);
    return Cnt(v, n, flip);
}
inline Cnt mul(Cnt a, Cnt b, double v, bool div)
{
    if (is_const(a) && is_const(b)) return Cnt(v);
    if (!div && ((is_const(a) && a.v == 0.0) || (is_const(b) && b.v == 0.0))) return Cnt(0.0);
    if (is_const(b) && (b.v == 1.0 || b.v == -1.0)) return b.v < 0 ? -a : a;
    if (!div && is_const(a) && (a.v == 1.0 || a.v == -1.0)) return a.v < 0 ? -b : b;
    // signs factor out of products and quotients; a constant operand is
    // keyed by its magnitude
    const bool flip = (a.neg != b.neg) != ((is_const(a) && a.v < 0) != (is_const(b) && b.v < 0));
    int ia = a.id, ib = b.id;
    long long ca = 0, cb = 0;
    if (is_const(a)) { double m = std::fabs(a.v); std::memcpy(&ca, &m, 8); ia = -1000000000 - (int)(ca % 1000000007ll % 1000000000); }
    if (is_const(b)) { double m = std::fabs(b.v); std::memcpy(&cb, &m, 8); ib = -1000000000 - (int)(cb % 1000000007ll % 1000000000); }
    if (!div && ia > ib) std::swap(ia, ib);
    const int n = cnt::make(div ? cnt::DIV : cnt::MUL, 0, ia, false, ib, false);
    return Cnt(v, n, flip);
}
inline Cnt trans(int sub, Cnt a, double v)
{
    if (is_const(a)) return Cnt(v);
    return Cnt(v, cnt::make(cnt::TRANS, sub, a.id, a.neg, -1, false));
}
inline Cnt operator+(Cnt a, Cnt b) { return add(a, b, a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { return add(a, -b, a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { return mul(a, b, a.v * b.v, false); }
inline Cnt operator/(Cnt a, Cnt b) { return mul(a, b, a.v / b.v, true); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v), a.id, false); }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }
inline Cnt sqrt(Cnt a) { return trans(1, a, std::sqrt(a.v)); }
inline Cnt exp(Cnt a) { return trans(2, a, std::exp(a.v)); }
inline Cnt expm1(Cnt a) { return trans(3, a, std::expm1(a.v)); }
inline Cnt erfc(Cnt a) { return trans(4, a, std::erfc(a.v)); }

struct Tally {
    long long add = 0, mul = 0, dv = 0, trans = 0;
};

// nodes created since `first` that the outputs depend on
static Tally live(size_t first, const std::vector<Cnt>& outs, double scale = 1.0)
{
    std::vector<char> seen(cnt::g.size(), 0);
    std::vector<int> stack;
    for (const Cnt& o : outs)
        if (o.id >= 0) stack.push_back(o.id);
    Tally t;
    while (!stack.empty()) {
        const int n = stack.back();
        stack.pop_back();
        if (n < 0 || seen[n]) continue;
        seen[n] = 1;
        if ((size_t)n < first) continue;
        const cnt::Node& d = cnt::g[n];
        (d.k == cnt::ADD ? t.add : d.k == cnt::MUL ? t.mul : d.k == cnt::DIV ? t.dv : t.trans) += 1;
        stack.push_back(d.a);
        stack.push_back(d.b);
    }
    t.add = (long long)(t.add / scale + 0.5);
    t.mul = (long long)(t.mul / scale + 0.5);
    t.dv = (long long)(t.dv / scale + 0.5);
    t.trans = (long long)(t.trans / scale + 0.5);
    return t;
}
static void emit(const char* name, Tally t, bool comma)
{
    printf("  \"%s\": {\"add\": %lld, \"mul\": %lld, \"div\": %lld, \"trans\": %lld, \"flops\": %lld}%s\n", name, t.add,
           t.mul, t.dv, t.trans, t.add + t.mul + t.dv + t.trans, comma ? "," : "");
}

static void smooth_state(Cnt* W, double s)
{
    const double rho = 1.0 + 0.1 * s, U = 0.3 - 0.05 * s, V = -0.2 + 0.04 * s, p = 1.0 + 0.07 * s;
    W[0] = data(rho); W[1] = data(rho * U); W[2] = data(rho * V); W[3] = data(p / 0.4 + 0.5 * rho * (U * U + V * V));
}

static void push4(std::vector<Cnt>& v, const Cnt* a)
{
    for (int k = 0; k < 4; ++k) v.push_back(a[k]);
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
            for (int k = 0; k < 4; ++k) Dk[q][k] = data(0.01 * (k + 1) * (q + 1));
        }
        cnt::memo.clear(); // merge common subexpressions within a unit only
        const size_t first = cnt::g.size();
        gks::face_recon<Cnt, 2, 8, Cnt>(Wk, Dk, Cnt(0.01), Cnt(gamma), true, [&](int q, int k, Cnt v) { o[q][k] = v; });
        std::vector<Cnt> outs;
        for (int q = 0; q < 7; ++q) push4(outs, o[q]);
        emit("face_row_2d", live(first, outs), true);
    }
    // ---- 2-D Gauss point (NS: mu > 0; and Euler), WENO-Z, averaged over the 3 points
    for (int ns = 1; ns >= 0; --ns) {
        Cnt rows[7][4][5];
        for (int r = 0; r < 5; ++r) {
            Cnt s[4];
            smooth_state(s, 0.05 * r);
            for (int k = 0; k < 4; ++k) {
                // the two non-equilibrium states differ from the equilibrium
                // value (as WENO-Z and linear reconstructions do)
                rows[0][k][r] = s[k];
                rows[3][k][r] = data(s[k].v * (1.0 + 1e-3 * (k + 1) + 2e-4 * r));
                rows[4][k][r] = data(s[k].v * (1.0 - 7e-4 * (k + 1) + 3e-4 * r));
                rows[1][k][r] = data(0.1 * (k + 1) + 0.003 * r); rows[2][k][r] = data(0.01 * (k + 2) + 0.001 * r);
                rows[5][k][r] = data(0.1 * (k + 1) + 0.002 * r); rows[6][k][r] = data(0.1 * (k + 1) - 0.002 * r);
            }
        }
        auto rv = [&](int q, int k, int r) { return rows[q][k][r]; };
        const gks::PointPar par = gks::point_par<2>(gamma, K2, ns ? 1e-4 : 0.0, 1e-3);
        cnt::memo.clear(); // merge common subexpressions within a unit only
        const size_t first = cnt::g.size();
        bool ok = true;
        std::vector<Cnt> all, s2;
        for (int G = 0; G < 3; ++G) {
            gks::PointIn<Cnt> in;
            gks::PointOut<Cnt> out;
            Cnt W0[4], Wl[4], Wr[4];
            gks::gp_inputs<Cnt, Cnt>(rv, G, Cnt(0.01), true, Cnt(gamma), in, W0, Wl, Wr);
            gks::NonEq<Cnt, 2> ne;
            ok = ok && gks::noneq_states<Cnt, 2>(Wl, Wr, Cnt(gamma), Cnt(K2), Cnt(par.iN), ne, in.Wlx, in.Wly, in.Wrx, in.Wry) &&
                 gks::gks_point<Cnt, 2, Cnt>(par, in, ne.Xs, ne, out);
            push4(all, out.FL); push4(all, out.FdL); push4(all, out.S0); push4(all, out.S1); push4(all, out.S2);
            push4(s2, out.FdL); push4(s2, out.S2);
        }
        if (!ok) {
            fprintf(stderr, "opcount: unexpected non-physical sample\n");
            return 1;
        }
        emit(ns ? "gauss_point_ns" : "gauss_point_euler", live(first, all, 3.0), true);
        emit(ns ? "gauss_point_ns_s2" : "gauss_point_euler_s2", live(first, s2, 3.0), true);
    }
    // ---- 1-D face, 8th order, WENO-Z, Euler
    {
        Cnt Wk[4][4], Dk[4][4], o[7][4];
        for (int q = 0; q < 4; ++q) {
            smooth_state(Wk[q], 0.1 * q);
            Wk[q][2] = 0.0;
            Wk[q][3] = data(1.0 / 0.4 + 0.5 * Wk[q][1].v * Wk[q][1].v / Wk[q][0].v);
            for (int k = 0; k < 4; ++k) Dk[q][k] = k == 2 ? Cnt(0.0) : data(0.01 * (k + 1) * (q + 1));
        }
        cnt::memo.clear(); // merge common subexpressions within a unit only
        const size_t first = cnt::g.size();
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
        const gks::PointPar par = gks::point_par<1>(gamma, K1, 0.0, 1e-3);
        ok = ok && gks::noneq_states<Cnt, 1>(o[3], o[4], Cnt(gamma), Cnt(K1), Cnt(par.iN), ne, in.Wlx, in.Wly, in.Wrx, in.Wry);
        ok = ok && gks::gks_point<Cnt, 1, Cnt>(par, in, ne.Xs, ne, out);
        if (!ok) {
            fprintf(stderr, "opcount: unexpected non-physical sample\n");
            return 1;
        }
        // 1-D state slots 0, 1, 3 (slot 2 is the absent v-momentum)
        std::vector<Cnt> all, s2;
        for (int k : {0, 1, 3}) {
            for (const Cnt* a : {out.FL, out.FdL, out.S0, out.S1, out.S2}) all.push_back(a[k]);
            s2.push_back(out.FdL[k]);
            s2.push_back(out.S2[k]);
        }
        emit("face_1d", live(first, all), true);
        emit("face_1d_s2", live(first, s2), false);
    }
    printf("}\n");
    return 0;
}
