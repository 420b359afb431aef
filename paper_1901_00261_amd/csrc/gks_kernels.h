// gks_kernels.h -- HIP kernels of the compact gas-kinetic scheme for gfx950.
//
// Data layout in HBM (all FP64, structure of arrays so that consecutive
// threads touch consecutive addresses):
//   1-D (batched): W[buf][3][Ntot], Wx[buf][3][Ntot]; problem p owns cells
//     coff_p .. coff_p + nx_p - 1.  Two buffers: W^n and the buffer that
//     receives W* and then W^{n+1} (the step commits by flipping `cur`, so a
//     failing step leaves W^n untouched).
//   2-D (one problem): W[buf][4][ny][nx], Wx, Wy alike.
//   Face arrays: 1-D [3][F] with F = sum_p (nx_p + 1) (the MSMD partial of
//     the face values only; fluxes stay in LDS); 2-D x faces
//     [4][ny][nx+1], y faces [4][ny+1][nx]; face-row reconstructions
//     [28][rows][faces].
// Ghost cells are never stored: stencil gathers map indices through the
// boundary condition (periodic wrap; extrapolation = copy of the boundary
// cell with the normal slope set to zero; reflecting wall = mirror image).
#pragma once

#include "gks_math.h"

namespace gks {
// Multiply-adds are contracted into FMAs only within one statement, so a
// function rounds the same way wherever it is inlined (the single-lane,
// lane-pair and two-kernel forms of the batched 1-D step agree bit for bit).
#pragma clang fp contract(on)

struct ProbParam {
    int nx, ny;
    long long coff; // first cell (1-D batching)
    long long foff; // first face (1-D batching)
    double dx, dy, gamma, K, mu, cfl, dt_fixed, t_end;
    int order, recon, bc[4];
    double xlo, ylo;
    double bstate[4][2][4]; // inflow states A, B per side (conservative, 4 slots)
    double bsplit[4][2];    // split sides: switch position at t = 0 and its speed
    int bbeyond[4];         // split sides: kind beyond the switch (inflow of B or reflecting)
};

// Side kinds as given (include/gks.h) and as resolved for one ghost cell.
constexpr int kBcPeriodic = 0, kBcExtrap = 1, kBcReflect = 2, kBcInflow = 3, kBcSplit = 4, kBcChar = 5;
constexpr int kResStateA = 3, kResStateB = 4;

struct ProbState {
    double t, dt;
    long long nsteps;
    unsigned long long smax; // bits of a non-negative double (max signal speed / dx)
    int active;              // still short of t_end and no error
    int err;                 // a non-physical state was met in this step
    int cur;                 // state slot holding W^n (2-D: slots 0, 1; 1-D: slots 0, 1, 2)
    int last;                // this step ends at t_end
};

struct Tile {
    int p;     // problem
    int start; // first face / cell of the tile
};

constexpr int kBlock1D = 128;

// Cell index through the boundary condition.  kind: 0 interior or
// periodic; 1 ghost of an extrapolated side (copy of the boundary cell,
// normal slope 0); 2 ghost of a reflecting wall (mirror image: the mirrored
// cell with its normal momentum negated, its normal slopes negated except
// that of the normal momentum); 3, 4 ghost holding the side's inflow state
// A or B (zero slopes; the index returned is the boundary cell, only so
// that loads stay in bounds); 5 characteristic ghost (1-D: built from the
// boundary cell, whose index is returned).
enum : int { kGhostNone = 0, kGhostCopy = 1, kGhostMirror = 2, kGhostStateA = 3, kGhostStateB = 4,
             kGhostChar = 5 };

// Resolved kind of the ghost cells of `side` at position pos along the side
// (cell-centre coordinate) at time t: a split side is inflow A below the
// moving switch point and its "beyond" kind past it.
__device__ __forceinline__ int resolve_side(const ProbParam& P, int side, double pos, double t)
{
    const int b = P.bc[side];
    if (b == kBcSplit)
        return pos < P.bsplit[side][0] + P.bsplit[side][1] * t ? kResStateA
                                                                 : (P.bbeyond[side] == kBcInflow ? kResStateB : kBcReflect);
    return b == kBcInflow ? kResStateA : b;
}

// One direction of the index map with a resolved side code (0 periodic,
// 1 extrapolated, 2 reflecting, 3/4 inflow A/B, 5 characteristic).
__device__ __forceinline__ int map_side(int c, int n, int code, int& kind)
{
    const bool lo = c < 0;
    if (code == kBcPeriodic) {
        kind = kGhostNone;
        return lo ? c + n : c - n;
    }
    if (code == kBcReflect) {
        kind = kGhostMirror;
        return lo ? -1 - c : 2 * n - 1 - c;
    }
    kind = code == kBcExtrap ? kGhostCopy : (code == kResStateA ? kGhostStateA : (code == kResStateB ? kGhostStateB : kGhostChar));
    return lo ? 0 : n - 1;
}
// Cell index of a 1-D stencil through the boundary conditions, with selects
// instead of branches (the boundary types are uniform, the side of the
// stencil per lane), so there is no divergent branch between a lane's
// stencil loads.
__device__ __forceinline__ int side_ghost_kind(int bc)
{
    return bc == kBcPeriodic ? kGhostNone
           : bc == kBcReflect ? kGhostMirror
           : bc == kBcInflow ? kGhostStateA
           : bc == kBcChar   ? kGhostChar
                             : kGhostCopy;
}
__device__ __forceinline__ int map_index_sel(int c, int n, int bc_lo, int bc_hi, int& kind)
{
    const int lm = bc_lo == 0 ? c + n : (bc_lo == 2 ? -1 - c : 0);
    const int lk = side_ghost_kind(bc_lo);
    const int hm = bc_hi == 0 ? c - n : (bc_hi == 2 ? 2 * n - 1 - c : n - 1);
    const int hk = side_ghost_kind(bc_hi);
    const bool lo = c < 0, hi = c >= n;
    kind = lo ? lk : (hi ? hk : kGhostNone);
    return lo ? lm : (hi ? hm : c);
}

// Faces of a 2-D direction with n cells that the interface kernel
// computes: with periodic ends the last face (index n) is the first one
// (the same stencil after the wrap, so the same result), so it is computed
// once and the cell update reads it as face 0.
__host__ __device__ inline int faces_computed(int n, int bc_lo) { return bc_lo == 0 ? n : n + 1; }

// Local-frame stencil entry (slot 1 = normal momentum, slot 2 = tangential
// momentum in 2-D) of a cell reached through map_index along the normal
// (kn) and the transverse (kt) direction: values w, normal slopes d.
__device__ __forceinline__ void ghost_frame(int kn, int kt, double (&w)[4], double (&d)[4])
{
    if (kn == kGhostCopy) d[0] = d[1] = d[2] = d[3] = 0.0;
    if (kn == kGhostMirror) {
        w[1] = -w[1];
        d[0] = -d[0]; d[2] = -d[2]; d[3] = -d[3];
    }
    if (kt == kGhostMirror) {
        w[2] = -w[2];
        d[2] = -d[2];
    }
}

// ghost_frame along the normal of a 1-D stencil (slot 2 unused), with selects
__device__ __forceinline__ void ghost_frame_1d(int kn, double (&w)[4], double (&d)[4])
{
    const bool copy = kn == kGhostCopy, mir = kn == kGhostMirror;
    w[1] = mir ? -w[1] : w[1];
    d[0] = copy ? 0.0 : (mir ? -d[0] : d[0]);
    d[1] = copy ? 0.0 : d[1];
    d[3] = copy ? 0.0 : (mir ? -d[3] : d[3]);
}

// Characteristic ghost of a 1-D side (w, d: the boundary cell's values and
// cell-width * slope on entry, the ghost's on return): fields with
// eigenvalue times outward normal out >= 0 leave the domain and are
// extended linearly over g cells, the others keep the boundary value with
// zero slope.  False if the boundary state is not physical.
__device__ __forceinline__ bool char_ghost_1d(double gamma, int g, int out, double (&w)[4], double (&d)[4])
{
    CharFrame<double, 1> fr;
    if (!fr.init(w, gamma)) return false;
    const double lam[4] = {fr.U - fr.c, fr.U, 0.0, fr.U + fr.c};
    double q[4], dq[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (a == 2) { q[a] = dq[a] = 0.0; continue; }
        double l[4];
        fr.left(a, l);
        const double v = l[0] * w[0] + l[1] * w[1] + l[3] * w[3];
        const double s = l[0] * d[0] + l[1] * d[1] + l[3] * d[3];
        const bool outgoing = out * lam[a] >= 0.0;
        q[a] = outgoing ? v + double(out * g) * s : v;
        dq[a] = outgoing ? s : 0.0;
    }
    fr.right(q, w);
    fr.right(dq, d);
    w[2] = d[2] = 0.0;
    return true;
}

// Two-stage MSMD combinations (Sec. 2.2) with the fused multiply-adds
// written out (the rounding does not depend on how a kernel is compiled):
//   msmd_half: a + dt/2 b + dt^2/8 c   (intermediate state / face value)
//   msmd_pred: a + dt b + dt^2/6 c     (first part of the full step)
//   msmd_corr: a + dt^2/3 c            (second-stage completion)
__device__ __forceinline__ double msmd_half(double a, double b, double c, double dt)
{
    return __builtin_fma(0.125 * dt * dt, c, __builtin_fma(0.5 * dt, b, a));
}
__device__ __forceinline__ double msmd_pred(double a, double b, double c, double dt)
{
    return __builtin_fma(dt * dt / 6.0, c, __builtin_fma(dt, b, a));
}
__device__ __forceinline__ double msmd_corr(double a, double c, double dt) { return __builtin_fma(dt * dt / 3.0, c, a); }

__device__ __forceinline__ double bits_to_double(unsigned long long b) { return __longlong_as_double((long long)b); }

// block-wide maximum of a non-negative value, one atomic per block
__device__ __forceinline__ void block_max_atomic(double v, unsigned long long* dst)
{
    __shared__ double red[16];
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wid = (threadIdx.x + threadIdx.y * blockDim.x) >> 6;
    const int nw = (blockDim.x * blockDim.y + 63) >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x + threadIdx.y * blockDim.x == 0) {
        double m = red[0];
        for (int w = 1; w < nw; ++w) m = fmax(m, red[w]);
        if (m > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(m));
    }
}

// block-wide maximum of a value (every thread receives it)
__device__ __forceinline__ double block_max(double v)
{
    __shared__ double red[16];
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wid = (threadIdx.x + threadIdx.y * blockDim.x) >> 6;
    const int nw = (blockDim.x * blockDim.y + 63) >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double m = red[0];
    for (int w = 1; w < nw; ++w) m = fmax(m, red[w]);
    return m;
}

// Workgroups are dispatched round-robin over the 8 XCDs (bid % 8), each with
// its own L2.  Give every XCD a contiguous range of tiles (a band of tile
// rows) so that the stencil neighbours of a tile are cached in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb)
{
    const int x = bid & 7, l = bid >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + l;
}

// 2-D tile coordinates of this workgroup (grid launched 1-D, gx tiles per row)
__device__ __forceinline__ void tile_xy(int gx, int& tx, int& ty)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    ty = t / gx;
    tx = t - ty * gx;
}

// ---------------------------------------------------------------------------
// Reconstruction at one face from a 4-cell stencil (local frame, slot 1 =
// normal velocity).  Wk/Dk: cell averages and cell-width * normal slopes of
// cells i-1..i+2.  emit(q, k, value) receives, in the local frame: q = 0 W0,
// 1 dn W0 (per unit length), 2 dnn W0, 3 Wl, 4 Wr, 5 dn Wl, 6 dn Wr.
// Non-physical WENO states fall back to the adjacent cell average.
// Types: D the stencil data and the emitted values; T the compact and WENO-Z
// arithmetic (on differences from the cell left of the face, formed in D);
// F the characteristic frame and the projections (FP32 in the mixed path).
// ---------------------------------------------------------------------------
// SPLIT = 2: a lane pair shares the face; the lane of the given side (0: the
// left state, 1: the right state, as the left state of the mirrored stencil)
// runs the WENO-Z of its side only and takes the other side from its
// partner.  SPLIT = 1: one lane runs both sides.  Both forms round alike:
// every multiply-add is contracted within its own statement (the fp
// contract pragma at the top of these headers), so the contraction does not
// depend on the code around it.
template <typename T, int DIM, int ORDER, typename D = double, typename F = D, int SPLIT = 1, typename Emit>
GKS_HD bool face_recon(const D (&Wk)[4][4], const D (&Dk)[4][4], D h, D gamma, bool weno, Emit&& emit, int side = 0)
{
    // outputs in O: FP32 when the frame is FP32 (the FP32-mixed path stores
    // them as FP32), otherwise D
    using O = std::conditional_t<std::is_same_v<F, float>, float, D>;
    const D ih = D(1) / h;
    const O iho = O(ih);
    // offsets from the cell left of the face keep the differences exact
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (DIM == 1 && k == 2) {
#pragma unroll
            for (int q = 0; q < 7; ++q) emit(q, k, O(0));
            continue;
        }
        const D base = Wk[1][k];
        const O baseo = O(base);
        T w[4], d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) { w[q] = T(Wk[q][k] - base); d[q] = T(Dk[q][k]); }
        T v, vx, vxx;
        linear_recon<T, ORDER>(w, d, v, vx, vxx);
        emit(0, k, baseo + O(v));
        emit(1, k, O(vx) * iho);
        emit(2, k, O(vxx) * iho * iho);
        if (!weno) {
            emit(3, k, baseo + O(v));
            emit(4, k, baseo + O(v));
            emit(5, k, O(vx) * iho);
            emit(6, k, O(vx) * iho);
        }
    }
    if (!weno) return true;
    // characteristic frame at the mean of the two interface cells
    F Wm[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) Wm[k] = F(D(0.5) * (Wk[1][k] + Wk[2][k]));
    CharFrame<F, DIM> fr;
    if (!fr.init(Wm, F(gamma))) return false;
    F ql[4], qr[4], qlx[4], qrx[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (DIM == 1 && a == 2) { ql[a] = qr[a] = qlx[a] = qrx[a] = F(0); continue; }
        F l[4];
        fr.left(a, l);
        T w[4], d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            F sw = F(0), sd = F(0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sw += l[k] * F(Wk[q][k] - Wk[1][k]);
                sd += l[k] * F(Dk[q][k]);
            }
            w[q] = T(sw);
            d[q] = T(sd);
        }
        T vl, dl, vr, dr;
        if constexpr (SPLIT == 1) {
            weno_left<T, ORDER>(w, d, vl, dl);
            weno_right<T, ORDER>(w, d, vr, dr);
        } else {
            // weno_right(w, d) is weno_left of the mirrored stencil with
            // the derivative negated
            T ws[4], ds[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ws[q] = side ? w[3 - q] : w[q];
                ds[q] = side ? -d[3 - q] : d[q];
            }
            T v, dd;
            weno_left<T, ORDER>(ws, ds, v, dd);
            const T pv = pair_swap(v), pd = pair_swap(dd);
            vl = side ? pv : v;
            dl = side ? pd : dd;
            vr = side ? v : pv;
            dr = -(side ? dd : pd);
        }
        ql[a] = F(vl); qlx[a] = F(dl); qr[a] = F(vr); qrx[a] = F(dr);
    }
    F Wlf[4], Wrf[4], Wlxf[4], Wrxf[4];
    fr.right(ql, Wlf);
    fr.right(qr, Wrf);
    fr.right(qlx, Wlxf);
    fr.right(qrx, Wrxf);
    O Wl[4], Wr[4], Wlx[4], Wrx[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Wl[k] = O(Wlf[k]) + O(Wk[1][k]);
        Wr[k] = O(Wrf[k]) + O(Wk[1][k]);
        Wlx[k] = O(Wlxf[k]);
        Wrx[k] = O(Wrxf[k]);
    }
    const bool okl = physical<O>(Wl, O(gamma), DIM), okr = physical<O>(Wr, O(gamma), DIM);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        emit(3, k, okl ? Wl[k] : O(Wk[1][k]));
        emit(4, k, okr ? Wr[k] : O(Wk[2][k]));
        emit(5, k, Wlx[k] * iho);
        emit(6, k, Wrx[k] * iho);
    }
    return true;
}

// ---------------------------------------------------------------------------
// Per-problem step bookkeeping.
//   commit = 1: the step just run is accepted (W^{n+1} becomes the state:
//               slot cur + nslot - 1 modulo nslot, so the next slot with two
//               slots and the slot after the half-step state with three;
//               advance t) or, after an error, the problem stops with W^n kept.
//   Then the next dt follows from the maximum signal speed of the state.
// ---------------------------------------------------------------------------
// Returns true when the problem stops here (error or t_end reached).
__device__ __forceinline__ bool finish_problem(const ProbParam& P, ProbState& S, int commit, int nslot)
{
    if (!S.active) return false;
    if (S.err) {
        S.active = 0;
        return true;
    }
    if (commit) {
        S.cur = S.cur == 0 ? nslot - 1 : S.cur - 1;
        S.t = S.last ? P.t_end : S.t + S.dt;
        S.nsteps += 1;
    }
    const double smax = bits_to_double(S.smax);
    S.smax = 0ull;
    if (!(S.t < P.t_end)) {
        S.active = 0;
        return true;
    }
    double dt = P.dt_fixed > 0.0 ? P.dt_fixed : P.cfl / smax;
    int last = 0;
    if (S.t + dt >= P.t_end - 1e-9 * dt) {
        dt = P.t_end - S.t;
        last = 1;
    }
    S.dt = dt;
    S.last = last;
    return false;
}

// one thread per problem (initial dt, and the 2-D step); ctr: work counters
// of the batched 1-D kernels, reset here (null for 2-D); nslot: state slots
__global__ void finish_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS, int nprob, int commit,
                              unsigned* __restrict__ ctr, int nslot)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (ctr && p < 3) ctr[p] = 0u;
    if (p < nprob) finish_problem(PP[p], PS[p], commit, nslot);
}

// Work list of the next step: the items of the problems still active, in
// problem order, built by one workgroup of NT threads that scans the
// problems in chunks (scan: NT ints of LDS).  first[p], count[p]: problem
// p's items in the full list.  Writes act[0..n) and *nact.
template <int NT>
__device__ void compact_items_block(const ProbState* __restrict__ PS, int nprob, const Tile* __restrict__ all,
                                    const int* __restrict__ first, const int* __restrict__ count,
                                    Tile* __restrict__ act, int* __restrict__ nact, int* scan)
{
    const int t = threadIdx.x;
    int base = 0;
    for (int p0 = 0; p0 < nprob; p0 += NT) {
        const int p = p0 + t;
        const int c = (p < nprob && PS[p].active) ? count[p] : 0;
        scan[t] = c;
        __syncthreads();
        for (int off = 1; off < NT; off <<= 1) { // inclusive scan
            const int v = t >= off ? scan[t - off] : 0;
            __syncthreads();
            scan[t] += v;
            __syncthreads();
        }
        const int dst = base + scan[t] - c;
        for (int i = 0; i < c; ++i) act[dst + i] = all[first[p] + i];
        base += scan[NT - 1];
        __syncthreads(); // scan[] reuse by the next chunk
    }
    if (t == 0) *nact = base;
}

constexpr int kCompactThreads = 256;
__global__ void __launch_bounds__(kCompactThreads) compact_items_kernel(const ProbState* __restrict__ PS, int nprob,
                                                                        const Tile* __restrict__ all,
                                                                        const int* __restrict__ first,
                                                                        const int* __restrict__ count,
                                                                        Tile* __restrict__ act, int* __restrict__ nact)
{
    __shared__ int scan[kCompactThreads];
    compact_items_block<kCompactThreads>(PS, nprob, all, first, count, act, nact, scan);
}

// The four stencil cells of face f of a 1-D problem through its boundary
// conditions: values and dx-scaled slopes (slot 2 zero), all 24 loads issued
// together.  Wb, Xb: the problem's first cell in the state and slope slots
// (component stride Ntot).  False when a characteristic ghost cell has no
// physical state.
__device__ __forceinline__ bool gather_face_1d(const ProbParam& P, const double* Wb, const double* Xb, long long Ntot,
                                               int f, double (&Wk)[4][4], double (&Dk)[4][4])
{
    int kind[4], c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = map_index_sel(f - 2 + q, P.nx, P.bc[0], P.bc[1], kind[q]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        Wk[q][0] = Wb[c[q]]; Wk[q][1] = Wb[Ntot + c[q]]; Wk[q][2] = 0.0; Wk[q][3] = Wb[2 * Ntot + c[q]];
        Dk[q][0] = Xb[c[q]]; Dk[q][1] = Xb[Ntot + c[q]]; Dk[q][2] = 0.0; Dk[q][3] = Xb[2 * Ntot + c[q]];
    }
    bool gok = true;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int k = 0; k < 4; ++k) Dk[q][k] *= P.dx;
        ghost_frame_1d(kind[q], Wk[q], Dk[q]);
        const int cq = f - 2 + q, side = cq < 0 ? 0 : 1;
        if (kind[q] == kGhostStateA) {
            const double* st = P.bstate[side][0];
            Wk[q][0] = st[0]; Wk[q][1] = st[1]; Wk[q][3] = st[3];
            Dk[q][0] = Dk[q][1] = Dk[q][3] = 0.0;
        } else if (kind[q] == kGhostChar) {
            gok = gok && char_ghost_1d(P.gamma, cq < 0 ? -cq : cq - P.nx + 1, side == 0 ? -1 : 1, Wk[q], Dk[q]);
        }
    }
    return gok;
}

// Cell c (global index) of a 1-D problem at the end of stage STAGE, from the
// values fv(q, k, s) of its left (s = 0) and right (s = 1) faces, q = 0 the
// flux F^L, 1 its time derivative, 2 the face state W_f (component k of 3),
// and its value wc(k) (stage 1: W^n; stage 2: the partial PW): writes
// W (slot wr), W_x and, in stage 1, PW.  Returns the cell's signal speed
// over dx after stage 2, flagging a non-physical state (0 then, and after
// stage 1).
template <int STAGE, typename FV, typename CV>
__device__ __forceinline__ double update_cell_1d(const ProbParam& P, ProbState& S, long long c, int wr, double dt,
                                                 double idx, const FV& fv, const CV& wc, double* __restrict__ W,
                                                 double* __restrict__ Wx, double* __restrict__ PW, long long Ntot)
{
    double wn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double dL = -(fv(1, k, 1) - fv(1, k, 0)) * idx;
        const double slope = (fv(2, k, 1) - fv(2, k, 0)) * idx;
        if (STAGE == 1) {
            const double L = -(fv(0, k, 1) - fv(0, k, 0)) * idx;
            const double w = wc(k);
            W[((size_t)wr * 3 + k) * Ntot + c] = msmd_half(w, L, dL, dt);
            PW[k * Ntot + c] = msmd_pred(w, L, dL, dt);
        } else {
            wn[k] = msmd_corr(wc(k), dL, dt);
            W[((size_t)wr * 3 + k) * Ntot + c] = wn[k];
        }
        Wx[((size_t)wr * 3 + k) * Ntot + c] = slope;
    }
    if (STAGE == 1) return 0.0;
    const double rho = wn[0], U = wn[1] / rho;
    const double p = (P.gamma - 1.0) * (wn[2] - 0.5 * rho * U * U);
    if (!(rho > 0.0) || !(p > 0.0)) {
        atomicOr(&S.err, 1);
        return 0.0;
    }
    return (fabs(U) + sqrt(P.gamma * p / rho)) * idx;
}

// Commit of a 1-D step by one workgroup: the step for every problem, the
// next dt, the counters reset and, when a problem has stopped, the work
// list rebuilt.
template <int BLK>
__device__ __forceinline__ void commit_step_block(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS,
                                                  int nprob, unsigned* __restrict__ ctr, const Tile* __restrict__ all,
                                                  const int* __restrict__ first, const int* __restrict__ count,
                                                  Tile* items, int* nitems_p)
{
    __shared__ int sh_stopped;
    __shared__ int sh_scan[BLK];
    const int t = threadIdx.x;
    if (t == 0) sh_stopped = 0;
    __syncthreads();
    bool stopped = false;
    for (int p = t; p < nprob; p += BLK) stopped |= finish_problem(PP[p], PS[p], 1, 3);
    if (stopped) atomicOr(&sh_stopped, 1);
    if (t < 3) ctr[t] = 0u;
    __syncthreads();
    // the list changes only when a problem has stopped; its scan reads the
    // problems' states in the order in which this workgroup's threads wrote
    // them (thread t: problems t, t + BLK, ...), so no fence is needed
    if (sh_stopped) compact_items_block<BLK>(PS, nprob, all, first, count, items, nitems_p, sh_scan);
}

// ---------------------------------------------------------------------------
// Batched 1-D: one launch per MSMD stage for all problems.  A work item is
// a tile of BLK-1 cells of one problem; the workgroup computes the BLK faces
// bounding it (the last face of a tile is also the first face of the next
// and is computed by both, bit-identically), keeps the face results in LDS
// and updates its cells.  Workgroups take items from a device counter until
// the list is exhausted, so the same kernel runs persistent (a few
// workgroups per CU) or as a plain grid (one workgroup per item); every
// workgroup reaches the exit.  The item list holds only the problems still
// active; its length is read from device memory, and workgroups beyond it
// leave at once.  commit1d_kernel, launched after the second stage, commits
// the step for every problem, resets the counters and, when a problem has
// stopped, rebuilds the list for the next step.  Faces owned by the tile
// (all but its last face, plus the problem's last face) carry the MSMD
// partial Pf from stage 1 to stage 2.
// ---------------------------------------------------------------------------
template <typename T, int STAGE, int BLK, int SPLIT = 1>
__global__ void __launch_bounds__(BLK, sizeof(T) == 4 ? 2 : 1) stage1d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS,
                                                      Tile* items, int* nitems_p,
                                                      unsigned* __restrict__ ctr, double* __restrict__ W,
                                                      double* __restrict__ Wx, double* __restrict__ PW,
                                                      double* __restrict__ Pf, long long Ntot, long long F)
{
    __shared__ double sh_FL[3][BLK], sh_FdL[3][BLK], sh_Wf[3][BLK];
    __shared__ double sh_cell[3][BLK], sh_face[3][BLK]; // the item's staged cell and face values
    __shared__ int sh_item;
    const int t = threadIdx.x;
    const int nitems = *nitems_p;
    // Only the first min(grid, items) workgroups take part (the grid is
    // sized for the full list; in a run's tail most problems have stopped):
    // the others leave before touching a counter.
    const int nwg = min((int)gridDim.x, nitems);
    if ((int)blockIdx.x >= nwg) return;
    // A workgroup's first item is its own index; each later one comes from
    // the counter (offset by the participants), requested as the previous
    // item starts, so that the atomic's latency hides behind that item.
    auto advance = [&](int n) {
        if (t == 0) sh_item = n;
        __syncthreads();
        const int v = sh_item;
        __syncthreads();
        return v;
    };
    int nxt = 0;
    for (int it = blockIdx.x; it < nitems; it = advance(nxt)) {
        if (t == 0) nxt = nwg + (int)atomicAdd(&ctr[STAGE - 1], 1u);
        const Tile tl = items[it];
        const ProbParam& P = PP[tl.p];
        ProbState& S = PS[tl.p];
        if (!S.active) continue; // uniform over the workgroup
        // state slots: stage 1 reads W^n (slot cur) and writes W^{n+1/2} to
        // the next slot; stage 2 reads W^{n+1/2} and writes W^{n+1} to the
        // third, so no item overwrites values a neighbouring item's stencil
        // still reads in the same launch, and W^n survives a failed step
        const int cur = S.cur, half = cur == 2 ? 0 : cur + 1, next = cur == 0 ? 2 : cur - 1;
        const int rd = STAGE == 1 ? cur : half, wr = STAGE == 1 ? half : next;
        const double dt = S.dt;
        // The item's values that the end of the stage needs (stage 1: W^n of
        // its cells; stage 2: the partials PW of its cells and Pf of its
        // faces) are copied into LDS with direct-to-LDS loads issued with the
        // stencil loads, so their latency overlaps.  Each wave copies its own
        // lanes' values (dword copies: lane l moves half l & 1 of value
        // l >> 1 of a 32-value run), so no other wave waits for them;
        // indices are clamped into the problem (values of lanes without a
        // cell or face are not used).
        {
            const int wv = t & ~63, l = t & 63;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int v = wv + 32 * c + (l >> 1);
                const long long cell = P.coff + min(tl.start + v, P.nx - 1);
                const long long face = P.foff + min(tl.start + v, P.nx);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double* src = STAGE == 1 ? W + ((size_t)cur * 3 + k) * Ntot + cell : PW + k * Ntot + cell;
                    __builtin_amdgcn_global_load_lds((const void*)((const char*)src + (l & 1) * 4),
                                                     (__attribute__((address_space(3))) void*)&sh_cell[k][wv + 32 * c],
                                                     4, 0, 0);
                    if (STAGE == 2)
                        __builtin_amdgcn_global_load_lds((const void*)((const char*)(Pf + k * F + face) + (l & 1) * 4),
                                                         (__attribute__((address_space(3))) void*)&sh_face[k][wv + 32 * c],
                                                         4, 0, 0);
                }
            }
        }
        // ---- faces c0 .. c0 + NF - 1 (NF = BLK / SPLIT: with SPLIT = 2 the
        // lanes 2j and 2j + 1 share face j, one WENO-Z side and one
        // non-equilibrium state each)
        constexpr int NF = BLK / SPLIT;
        const int j = t / SPLIT, side = t % SPLIT;
        const int f = tl.start + j;
        if (f <= P.nx) {
            double Wk[4][4], Dk[4][4];
            const bool gok = gather_face_1d(P, W + (size_t)rd * 3 * Ntot + P.coff, Wx + (size_t)rd * 3 * Ntot + P.coff,
                                            Ntot, f, Wk, Dk);
            // face reconstruction emitted in T (the FP32-mixed path stores
            // and evaluates the interface point in FP32)
            T o[7][4];
            auto put = [&](int q, int k, auto v) { o[q][k] = T(v); };
            bool ok = gok && ((P.order == 8) ? face_recon<T, 1, 8, double, T, SPLIT>(Wk, Dk, P.dx, P.gamma, P.recon != 0, put, side)
                                             : face_recon<T, 1, 6, double, T, SPLIT>(Wk, Dk, P.dx, P.gamma, P.recon != 0, put, side));
            PointIn<T> in;
            PointOut<T> out;
            NonEq<T, 1, T> ne;
            const PointPar par = point_par<1>(P.gamma, P.K, P.mu, dt);
            if (ok) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    in.W0x[k] = o[1][k]; in.W0xx[k] = o[2][k];
                    in.W0y[k] = in.W0xy[k] = in.W0yy[k] = T(0);
                    in.Wlx[k] = o[5][k]; in.Wrx[k] = o[6][k];
                    in.Wly[k] = in.Wry[k] = T(0);
                }
                if constexpr (SPLIT == 1) {
                    ok = noneq_states<T, 1, T>(o[3], o[4], T(P.gamma), T(P.K), T(par.iN), ne, in.Wlx, in.Wly, in.Wrx,
                                               in.Wry);
                } else {
                    // this lane's state (selected element by element, so that
                    // the arrays stay in registers), then the partner's share
                    T Ws[4], Wn[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) { Ws[k] = side ? o[4][k] : o[3][k]; Wn[k] = side ? in.Wrx[k] : in.Wlx[k]; }
                    NeSide<T, 1, T> own, l, r;
                    const bool oko = noneq_side<T, 1, T>(Ws, side, T(P.gamma), T(P.K), T(par.iN), own, Wn, in.Wly);
                    const bool okp = __builtin_amdgcn_update_dpp(0, (int)oko, 0xB1, 0xF, 0xF, false) != 0;
                    ok = oko && okp;
                    // left share first, whichever lane holds it
                    auto pick = [&](T mine, T& lv, T& rv) {
                        const T other = pair_swap(mine);
                        lv = side ? other : mine;
                        rv = side ? mine : other;
                    };
                    pick(own.p, l.p, r.p);
                    pick(own.rs, l.rs, r.rs);
                    pick(own.rt, l.rt, r.rt);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        pick(own.h0[k], l.h0[k], r.h0[k]);
                        pick(own.h1[k], l.h1[k], r.h1[k]);
                        pick(own.h2[k], l.h2[k], r.h2[k]);
                        pick(own.h3[k], l.h3[k], r.h3[k]);
                    }
                    noneq_combine<T, 1, T>(l, r, ne);
                }
            }
            if (ok) ok = gks_point<T, 1, T>(par, in, P.recon ? ne.Xs : o[0], ne, out);
            if (!ok) {
                atomicOr(&S.err, 1);
#pragma unroll
                for (int k = 0; k < 4; ++k) out.FL[k] = out.FdL[k] = out.S0[k] = out.S1[k] = out.S2[k] = T(0);
            }
            const bool own = (j < NF - 1) || (f == P.nx);
            const long long g = P.foff + f;
            const int slot[3] = {0, 1, 3};
            if (side == 0) // both lanes of a pair hold the same results
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int sl = slot[k];
                    sh_FdL[k][j] = double(out.FdL[sl]);
                    if (STAGE == 1) {
                        const double s0 = double(out.S0[sl]), s1 = double(out.S1[sl]), s2 = double(out.S2[sl]);
                        sh_FL[k][j] = double(out.FL[sl]);
                        sh_Wf[k][j] = msmd_half(s0, s1, s2, dt);
                        if (own) Pf[k * F + g] = msmd_pred(s0, s1, s2, dt);
                    } else {
                        sh_Wf[k][j] = msmd_corr(sh_face[k][j], double(out.S2[sl]), dt);
                    }
                }
        }
        __syncthreads();
        // ---- cells c0 .. c0 + NF - 2
        const int i = tl.start + t;
        const bool live = (t < NF - 1) && (i < P.nx);
        const double idx = 1.0 / P.dx;
        const double sp = live ? update_cell_1d<STAGE>(
                                     P, S, P.coff + i, wr, dt, idx,
                                     [&](int q, int k, int s) {
                                         return q == 0 ? sh_FL[k][t + s] : (q == 1 ? sh_FdL[k][t + s] : sh_Wf[k][t + s]);
                                     },
                                     [&](int k) { return sh_cell[k][t]; }, W, Wx, PW, Ntot)
                               : 0.0;
        if (STAGE == 2) block_max_atomic(sp, &S.smax);
        __syncthreads(); // LDS reuse by the next item
    }
}

// ---------------------------------------------------------------------------
// Batched 1-D, two-kernel form of a stage: the fused kernel split after the
// face reconstruction, over the same 255-cell work items (one workgroup per
// item, workgroups beyond the active items leaving at once): face1d_kernel
// reconstructs the item's own faces into HBM, pointcell1d_kernel evaluates
// the interface point of every face of the item and updates its cells.
// Each fits in fewer registers than the fused kernel (FP64: 206 and 168
// against 366), so more waves share a SIMD.  The results are those of the
// fused kernel bit for bit.  Face buffer R1[21] (F faces, component stride
// F): quantity q (face_recon order) of component k in row 3 q + k',
// k' = 0, 1, 2 for the components rho, rho U, rho E (type T).
// ---------------------------------------------------------------------------
constexpr int kPhaseBlk = 256;

// First kernel of the two-kernel form: gather and reconstruction of the
// item's own faces (all but its last face, plus the problem's last face),
// stored in T.
template <typename T, int STAGE>
__global__ void __launch_bounds__(kPhaseBlk, 2)
    face1d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS, const Tile* __restrict__ items,
                  const int* __restrict__ nitems_p, const double* __restrict__ W, const double* __restrict__ Wx,
                  T* __restrict__ R1, long long Ntot, long long F)
{
    if ((int)blockIdx.x >= *nitems_p) return;
    const Tile tl = items[blockIdx.x];
    const ProbParam& P = PP[tl.p];
    ProbState& S = PS[tl.p];
    if (!S.active) return;
    const int j = threadIdx.x, f = tl.start + j;
    if (f > P.nx || (j == kPhaseBlk - 1 && f != P.nx)) return;
    const int cur = S.cur, rd = STAGE == 1 ? cur : (cur == 2 ? 0 : cur + 1);
    double Wk[4][4], Dk[4][4];
    const bool gok = gather_face_1d(P, W + (size_t)rd * 3 * Ntot + P.coff, Wx + (size_t)rd * 3 * Ntot + P.coff, Ntot, f,
                                    Wk, Dk);
    T* r = R1 + P.foff + f;
    auto put = [&](int q, int k, auto v) {
        if (k != 2) r[(q * 3 + (k == 3 ? 2 : k)) * F] = T(v);
    };
    const bool ok = gok && ((P.order == 8) ? face_recon<T, 1, 8, double, T>(Wk, Dk, P.dx, P.gamma, P.recon != 0, put)
                                           : face_recon<T, 1, 6, double, T>(Wk, Dk, P.dx, P.gamma, P.recon != 0, put));
    if (!ok) atomicOr(&S.err, 1);
}

// Second kernel of the two-kernel form: the interface point of every face
// of the item (its last face, owned by the next item, too, as in the fused
// kernel), the MSMD face values kept in LDS, then the item's cells; after
// stage 2 their signal speeds.
template <typename T, int STAGE>
__global__ void __launch_bounds__(kPhaseBlk, 3)
    pointcell1d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS, const Tile* __restrict__ items,
                       const int* __restrict__ nitems_p, const T* __restrict__ R1, double* __restrict__ W,
                       double* __restrict__ Wx, double* __restrict__ PW, double* __restrict__ Pf, long long Ntot,
                       long long F)
{
    __shared__ double sh_FL[3][kPhaseBlk], sh_FdL[3][kPhaseBlk], sh_Wf[3][kPhaseBlk];
    if ((int)blockIdx.x >= *nitems_p) return;
    const Tile tl = items[blockIdx.x];
    const ProbParam& P = PP[tl.p];
    ProbState& S = PS[tl.p];
    if (!S.active) return;
    const int j = threadIdx.x, f = tl.start + j;
    const double dt = S.dt;
    if (f <= P.nx) {
        const long long g = P.foff + f;
        T o[7][4];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            o[q][0] = R1[(q * 3) * F + g];
            o[q][1] = R1[(q * 3 + 1) * F + g];
            o[q][2] = T(0);
            o[q][3] = R1[(q * 3 + 2) * F + g];
        }
        PointIn<T> in;
        PointOut<T> out;
        NonEq<T, 1, T> ne;
        const PointPar par = point_par<1>(P.gamma, P.K, P.mu, dt);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            in.W0x[k] = o[1][k]; in.W0xx[k] = o[2][k];
            in.W0y[k] = in.W0xy[k] = in.W0yy[k] = T(0);
            in.Wlx[k] = o[5][k]; in.Wrx[k] = o[6][k];
            in.Wly[k] = in.Wry[k] = T(0);
        }
        bool ok = noneq_states<T, 1, T>(o[3], o[4], T(P.gamma), T(P.K), T(par.iN), ne, in.Wlx, in.Wly, in.Wrx, in.Wry);
        if (ok) ok = gks_point<T, 1, T>(par, in, P.recon ? ne.Xs : o[0], ne, out);
        if (!ok) {
            atomicOr(&S.err, 1);
#pragma unroll
            for (int k = 0; k < 4; ++k) out.FL[k] = out.FdL[k] = out.S0[k] = out.S1[k] = out.S2[k] = T(0);
        }
        const bool own = (j < kPhaseBlk - 1) || (f == P.nx);
        const int slot[3] = {0, 1, 3};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int sl = slot[k];
            sh_FdL[k][j] = double(out.FdL[sl]);
            if (STAGE == 1) {
                const double s0 = double(out.S0[sl]), s1 = double(out.S1[sl]), s2 = double(out.S2[sl]);
                sh_FL[k][j] = double(out.FL[sl]);
                sh_Wf[k][j] = msmd_half(s0, s1, s2, dt);
                if (own) Pf[k * F + g] = msmd_pred(s0, s1, s2, dt);
            } else {
                sh_Wf[k][j] = msmd_corr(Pf[k * F + g], double(out.S2[sl]), dt);
            }
        }
    }
    __syncthreads();
    const int i = tl.start + j;
    const bool live = j < kPhaseBlk - 1 && i < P.nx;
    const int cur = S.cur, half = cur == 2 ? 0 : cur + 1, next = cur == 0 ? 2 : cur - 1;
    const int wr = STAGE == 1 ? half : next;
    const double idx = 1.0 / P.dx;
    const long long c = P.coff + i;
    const double sp = live ? update_cell_1d<STAGE>(
                                 P, S, c, wr, dt, idx,
                                 [&](int q, int k, int s) {
                                     return q == 0 ? sh_FL[k][j + s] : (q == 1 ? sh_FdL[k][j + s] : sh_Wf[k][j + s]);
                                 },
                                 [&](int k) { return STAGE == 1 ? W[((size_t)cur * 3 + k) * Ntot + c] : PW[k * Ntot + c]; },
                                 W, Wx, PW, Ntot)
                           : 0.0;
    if (STAGE == 2) block_max_atomic(sp, &S.smax);
}

// The step's commit after the second stage of any form: one workgroup (the
// launch boundary orders it after the stage's writes, so no workgroup of
// the stage needs a device-wide fence or a done counter).
__global__ void __launch_bounds__(kPhaseBlk)
    commit1d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS, Tile* items, int* nitems_p,
                    unsigned* __restrict__ ctr, int nprob, const Tile* __restrict__ all, const int* __restrict__ first,
                    const int* __restrict__ count)
{
    commit_step_block<kPhaseBlk>(PP, PS, nprob, ctr, all, first, count, items, nitems_p);
}

// maximum signal speed of the current state (start of a run)
__global__ void __launch_bounds__(kBlock1D) signal1d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS,
                                                            const Tile* __restrict__ tiles, const double* __restrict__ W,
                                                            long long Ntot)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbParam& P = PP[tl.p];
    ProbState& S = PS[tl.p];
    const int i = tl.start + threadIdx.x;
    double s = 0.0;
    if (i < P.nx) {
        const long long c = P.coff + i;
        const double* Wb = W + (size_t)S.cur * 3 * Ntot;
        const double rho = Wb[c], U = Wb[Ntot + c] / rho;
        const double p = (P.gamma - 1.0) * (Wb[2 * Ntot + c] - 0.5 * rho * U * U);
        if (!(rho > 0.0) || !(p > 0.0)) S.err = 1;
        else s = (fabs(U) + sqrt(P.gamma * p / rho)) * (1.0 / P.dx); // as in the step kernels
    }
    block_max_atomic(s, &S.smax);
}

// Row stride of the 2-D row buffers (elements of size ES bytes: 8 in FP64,
// 4 in the FP32-mixed path): the row length rounded up to a multiple of 16
// bytes, so that rows and planes start on 16-byte boundaries (the interface
// kernel stages them with 16-byte copies).
__host__ __device__ constexpr int row_stride(int len, int ES = 8)
{
    return ES == 8 ? (len + 1) & ~1 : (len + 3) & ~3;
}

// Elements allocated past the end of a 2-D row buffer: the staging copies of
// the workgroups at the grid's far edges read up to three rows (of at most
// nx + 5 elements) plus one 128-element segment beyond the last plane, so
// every copy stays inside the allocation.
__host__ __device__ constexpr long long row_buffer_pad(int nx) { return 3ll * (nx + 5) + 128; }

// Elements of the row buffer of direction dir: 28 planes of A rows of
// stride row_stride(B, ES), plus the pad.
__host__ __device__ constexpr long long row_buffer_elems(int nx, int ny, int dir, int ES = 8)
{
    return 28ll * (dir == 0 ? ny + 4 : ny + 1) * row_stride(dir == 0 ? nx + 1 : nx + 4, ES) + row_buffer_pad(nx);
}

// ---------------------------------------------------------------------------
// 2-D.  DIR 0: x faces, DIR 1: y faces (local frame swaps slots 1 and 2).
// Face-row kernel: one thread per (face, transverse row incl. two ghost rows
// per side); stores the seven reconstructed vectors of face_recon.  ORDER
// (6 or 8) is the problem's, chosen at launch.
// Row buffer R[28][A][Bs], thread-x index b fastest, rows of B values
// stored with stride Bs = row_stride(B):
//   DIR 0: a = row + 2 (ny + 4 rows), b = face (nx + 1)
//   DIR 1: a = face (ny + 1), b = column + 2 (nx + 4)
// ---------------------------------------------------------------------------
template <typename T, int DIR, int ORDER>
__global__ void __launch_bounds__(256) row2d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS,
                                                    const double* __restrict__ W, const double* __restrict__ Wx,
                                                    const double* __restrict__ Wy, int stage, T* __restrict__ R)
{
    const ProbParam& P = PP[0];
    ProbState& S = PS[0];
    if (!S.active) return;
    const int nx = P.nx, ny = P.ny;
    const int nf = DIR == 0 ? nx + 1 : ny + 1;
    const int nt = DIR == 0 ? ny : nx;
    const int A = DIR == 0 ? nt + 4 : nf, B = DIR == 0 ? nf : nt + 4;
    // rows computed: the faces the interface kernel uses (faces_computed)
    const int nfc = faces_computed(nf - 1, DIR == 0 ? P.bc[0] : P.bc[2]);
    const int Ac = DIR == 0 ? A : nfc, Bc = DIR == 0 ? nfc : B;
    int tx, ty;
    tile_xy((Bc + blockDim.x - 1) / blockDim.x, tx, ty);
    const int b = tx * blockDim.x + threadIdx.x;
    const int a = ty * blockDim.y + threadIdx.y;
    if (a >= Ac || b >= Bc) return;
    const int face = DIR == 0 ? b : a;
    const int tr = (DIR == 0 ? a : b) - 2; // transverse index, -2 .. nt+1
    const int buf = stage == 1 ? S.cur : 1 - S.cur;
    const size_t plane = (size_t)nx * ny;
    const double* Wb = W + (size_t)buf * 4 * plane;
    const double* Nb = (DIR == 0 ? Wx : Wy) + (size_t)buf * 4 * plane;
    const double h = DIR == 0 ? P.dx : P.dy;
    double Wk[4][4], Dk[4][4];
    // time of this stage's data (time-dependent boundary states)
    const double tg = stage == 1 ? S.t : S.t + 0.5 * S.dt;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        // the stencil cell (xi, yj); ghosts map through the boundary
        // conditions, the y sides first (corner ghosts follow the y sides):
        // extrapolated rows / columns are copies (normal slope zero across
        // their own side), mirrored ones negate the momentum normal to their
        // side, inflow ghosts hold the side's state with zero slopes
        const int xi = DIR == 0 ? face - 2 + q : tr;
        const int yj = DIR == 0 ? tr : face - 2 + q;
        int ky = kGhostNone, yjm = yj;
        if (yj < 0 || yj >= ny)
            yjm = map_side(yj, ny, resolve_side(P, yj < 0 ? 2 : 3, P.xlo + (xi + 0.5) * P.dx, tg), ky);
        int kx = kGhostNone, xim = xi;
        if (ky >= kGhostStateA) xim = min(max(xi, 0), nx - 1);
        else if (xi < 0 || xi >= nx)
            xim = map_side(xi, nx, resolve_side(P, xi < 0 ? 0 : 1, P.ylo + (yjm + 0.5) * P.dy, tg), kx);
        const size_t cell = (size_t)yjm * nx + xim;
        double w[4], d[4];
        // local frame: normal momentum in slot 1, tangential in slot 2
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int g = (DIR == 1 && (k == 1 || k == 2)) ? 3 - k : k;
            w[k] = Wb[g * plane + cell];
            d[k] = h * Nb[g * plane + cell];
        }
        if (ky >= kGhostStateA || kx >= kGhostStateA) {
            const bool ys = ky >= kGhostStateA;
            const double* st = ys ? P.bstate[yj < 0 ? 2 : 3][ky - kGhostStateA] : P.bstate[xi < 0 ? 0 : 1][kx - kGhostStateA];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = st[(DIR == 1 && (k == 1 || k == 2)) ? 3 - k : k];
                d[k] = 0.0;
            }
            kx = kGhostNone;
            if (ys) ky = kGhostNone;
        }
        ghost_frame(DIR == 0 ? kx : ky, DIR == 0 ? ky : kx, w, d);
#pragma unroll
        for (int k = 0; k < 4; ++k) { Wk[q][k] = w[k]; Dk[q][k] = d[k]; }
    }
    // the 28 stores through a buffer resource: the lane's byte offset in a
    // plane as the 32-bit vector offset, the plane as a scalar offset (the
    // host guarantees row_buffer_elems(nx, ny, DIR, 8) * 8 < 2^32)
    const unsigned Bs = (unsigned)row_stride(B, sizeof(T));
    const unsigned rplane = (unsigned)A * Bs * (unsigned)sizeof(T);
    const unsigned voff = ((unsigned)a * Bs + (unsigned)b) * (unsigned)sizeof(T);
    const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)R, (short)0, (int)(unsigned)(row_buffer_elems(nx, ny, DIR, sizeof(T)) * sizeof(T)), 0x00020000);
    auto put = [&](int q, int k, auto v) {
        const unsigned so = (unsigned)(q * 4 + k) * rplane;
        using u32x2 = unsigned __attribute__((vector_size(8)));
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, double(v)), rsrc, voff, so, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, T(v)), rsrc, voff, so, 0);
    };
    const bool ok = face_recon<T, 2, ORDER, double, T>(Wk, Dk, h, P.gamma, P.recon != 0, put);
    if (!ok) S.err = 1;
}

// Gauss-point inputs at point g (0..2) of the 3-point rule: tangential
// linear 5th-order reconstruction of the equilibrium rows and of the
// derivatives of the non-equilibrium rows, tangential WENO-Z of the
// non-equilibrium values (with the positivity fallback to the face-row line
// value).  rv(q, k, r): quantity q (face_recon order), component k, row
// r = 0..4 (rows j-2..j+2).  Values in type D: W0 (linear), Wl, Wr.
//
// The inputs of component k come in two independent groups: gp_noneq_k
// forms the non-equilibrium values and derivatives (quantities 3-6 of
// face_recon), gp_equil_k the equilibrium value and derivatives
// (quantities 0-2); each reads only rv(., k, .), so a caller can stage the
// stencil one component at a time and form the second group after the
// non-equilibrium states have been evaluated.  gp_fallback then applies the
// positivity fallback, which reads the centre row of all four components.
template <typename T, typename D, typename Acc>
GKS_HD void gp_noneq_k(const Acc& rv, int g, int k, D iht, bool weno, PointIn<T>& in, D* Wl, D* Wr)
{
    D v5 = D(0), v6 = D(0), d3 = D(0), d4 = D(0);
    const D base = rv(0, k, 2);
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        const D c0 = tan_lin<D>(g, 0, r), c1 = tan_lin<D>(g, 1, r);
        v5 += c0 * rv(5, k, r);
        v6 += c0 * rv(6, k, r);
        d3 += c1 * (rv(3, k, r) - base);
        d4 += c1 * (rv(4, k, r) - base);
    }
    in.Wlx[k] = T(v5);
    in.Wrx[k] = T(v6);
    in.Wly[k] = T(d3 * iht);
    in.Wry[k] = T(d4 * iht);
    // both values formed first and stored once: stores to different arrays
    // in the two branches would otherwise be merged into one store through a
    // selected pointer, which keeps the arrays in scratch memory
    D wl, wr;
    if (weno) {
        D ql[5], qr[5];
#pragma unroll
        for (int r = 0; r < 5; ++r) { ql[r] = rv(3, k, r) - base; qr[r] = rv(4, k, r) - base; }
        D vl, vr;
        if constexpr (std::is_same_v<D, float>) {
            vl = tan_weno_f32(ql, g);
            vr = tan_weno_f32(qr, g);
        } else {
            tan_weno_pair<D>(ql, qr, g, vl, vr);
        }
        wl = base + vl;
        wr = base + vr;
    } else {
        // linear mode: both states are the equilibrium value
        D v0 = D(0);
#pragma unroll
        for (int r = 0; r < 5; ++r) v0 += tan_lin<D>(g, 0, r) * (rv(0, k, r) - base);
        wl = wr = base + v0;
    }
    Wl[k] = wl;
    Wr[k] = wr;
}

template <typename T, typename D, typename Acc>
GKS_HD void gp_equil_k(const Acc& rv, int g, int k, D iht, PointIn<T>& in, D* W0)
{
    D v0 = D(0), v1 = D(0), v2 = D(0), d0 = D(0), d1 = D(0), dd0 = D(0);
    const D base = rv(0, k, 2);
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        const D c0 = tan_lin<D>(g, 0, r), c1 = tan_lin<D>(g, 1, r), c2 = tan_lin<D>(g, 2, r);
        const D q0 = rv(0, k, r) - base;
        v0 += c0 * q0;
        d0 += c1 * q0;
        dd0 += c2 * q0;
        const D q1 = rv(1, k, r);
        v1 += c0 * q1;
        d1 += c1 * q1;
        v2 += c0 * rv(2, k, r);
    }
    W0[k] = base + v0;
    in.W0x[k] = T(v1);
    in.W0xx[k] = T(v2);
    in.W0y[k] = T(d0 * iht);
    in.W0xy[k] = T(d1 * iht);
    in.W0yy[k] = T(dd0 * iht * iht);
}

template <typename D, typename Acc>
GKS_HD void gp_fallback(const Acc& rv, bool weno, D gamma, D* Wl, D* Wr)
{
    if (weno) {
        if (!physical<D>(Wl, gamma, 2))
#pragma unroll
            for (int k = 0; k < 4; ++k) Wl[k] = rv(3, k, 2);
        if (!physical<D>(Wr, gamma, 2))
#pragma unroll
            for (int k = 0; k < 4; ++k) Wr[k] = rv(4, k, 2);
    }
}

template <typename T, typename D, typename Acc>
GKS_HD void gp_inputs(const Acc& rv, int g, D ht, bool weno, D gamma, PointIn<T>& in, D* W0, D* Wl, D* Wr)
{
    const D iht = D(1) / ht;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        gp_equil_k<T, D>(rv, g, k, iht, in, W0);
        gp_noneq_k<T, D>(rv, g, k, iht, weno, in, Wl, Wr);
    }
    gp_fallback<D>(rv, weno, gamma, Wl, Wr);
}

// Row-buffer reads through a buffer resource: 32-bit per-lane offsets for
// the five stencil rows, the quantity plane as a scalar offset.  The
// interface kernel uses it only for the rare positivity fallback.
template <typename S>
struct RowReader {
    __amdgpu_buffer_rsrc_t rsrc;
    unsigned voff[5];  // byte offset of row r (lane dependent)
    unsigned plane;    // bytes between quantity planes
    __device__ __forceinline__ S operator()(int q, int k, int r) const
    {
        if constexpr (sizeof(S) == 8) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff[r], (unsigned)(q * 4 + k) * plane, 0);
            return __builtin_bit_cast(S, v);
        } else {
            const auto v = __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff[r], (unsigned)(q * 4 + k) * plane, 0);
            return __builtin_bit_cast(S, v);
        }
    }
};

// Interface-kernel workgroup: 64 lanes along the contiguous index of the
// row buffer (x faces: the face; y faces: the transverse cell) times 4 waves
// (x faces: four transverse rows; y faces: four faces).  FP64: its LDS (the
// staged stencil and the Gauss sums) takes one workgroup per CU, one wave
// per SIMD; FP32-mixed: half the LDS, two workgroups per CU.
constexpr int kGpX = 64, kGpY = 4;

// LDS staging of the workgroup's stencil (elements of type S): slot k holds
// component k of the 7 quantities of face_recon over the rows the
// workgroup needs.  The waves copy it themselves, once, with 16-byte
// direct-to-LDS loads (no registers held); the three Gauss points then read
// it from LDS.
//   x faces: 8 transverse rows (4 waves + 4 stencil rows) x 64 faces, one
//            copy per row pair (FP64: lanes 0-31 the first row, 32-63 the
//            second; FP32: lanes 0-15 and 16-31, lanes 32-63 idle);
//   y faces: 4 face rows x 128 transverse entries, of which the 68 read (64
//            lanes + 4 stencil entries) are copied: one copy per row (FP64
//            lanes 0-33, FP32 lanes 0-16; the copies are bound by the memory
//            system's throughput, so the unread 60 entries are not fetched).
template <int DIR, typename S>
struct GpStage {
    static constexpr int rows = DIR == 0 ? kGpY + 4 : kGpY; // rows per quantity
    static constexpr int len = DIR == 0 ? kGpX : 2 * kGpX;   // elements per row
    static constexpr int elems = 7 * rows * len;
    static constexpr int copies = 7;                          // per wave and component
    static constexpr int per16 = 16 / (int)sizeof(S);         // elements per 16-byte lane copy
    // lanes taking part in one copy
    static constexpr int lanes = DIR == 0 ? 2 * kGpX / per16 : (kGpX + 4 + per16 - 1) / per16;
};

// Reader of a staged component: lane's row r of quantity q.
template <int DIR, typename S>
struct StageReader {
    const S* p; // slot + w * len + lane
    __device__ __forceinline__ S operator()(int q, int, int r) const
    {
        using G = GpStage<DIR, S>;
        return DIR == 0 ? p[(q * G::rows + r) * G::len] : p[q * G::rows * G::len + r];
    }
};

// Wave w's copies of one component into slot dst: x faces, row pair w of
// every quantity; y faces, its own face row of every quantity.  sofs: byte
// offset in the row buffer of the workgroup's first row of quantity 0 at
// this component; plane / rstride: bytes between quantity planes / rows;
// voff: the lane's byte offset within a copy.
template <int DIR, typename S>
__device__ __forceinline__ void stage_component(__amdgpu_buffer_rsrc_t rs, S* dst, unsigned sofs, unsigned plane,
                                                unsigned rstride, int w, unsigned voff)
{
    using G = GpStage<DIR, S>;
    const int row = DIR == 0 ? 2 * w : w;
    // lanes past G::lanes would copy entries that no lane reads
    if ((int)(threadIdx.x & 63) < G::lanes) {
#pragma unroll
        for (int q = 0; q < 7; ++q)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rs, (__attribute__((address_space(3))) void*)(dst + (q * G::rows + row) * G::len), 16, voff,
                sofs + (unsigned)(q * 4) * plane + (unsigned)row * rstride, 0, 0);
    }
}

// Wait until this wave's copies of components 0..K have landed (the 7 copies
// of each later component may still be in flight), then for the whole
// workgroup, whose waves share the x-face rows.
template <int K>
__device__ __forceinline__ void stage_wait()
{
    constexpr int n = 7 * (3 - K);
    static_assert(n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | 0x0F70); // vmcnt(n), other counters free
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Interface kernel.  T: the arithmetic and storage type of the face-row
// buffer, the staged stencil, the Gauss-point evaluation and the Gauss sums
// (double in FP64, float in the FP32-mixed path); the time-integration
// coefficients are FP64 in both, and so are the MSMD face partials written
// at the end.
template <typename T, int DIR, int STAGE>
__global__ void __launch_bounds__(kGpX * kGpY, sizeof(T) == 4 ? 2 : 1)
    gp2d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS, const T* __restrict__ R,
                double* __restrict__ FL, double* __restrict__ FdL, double* __restrict__ Wfs, double* __restrict__ Pf)
{
    const ProbParam& P = PP[0];
    ProbState& S = PS[0];
    if (!S.active) return;
    constexpr unsigned ES = sizeof(T);
    const int nx = P.nx, ny = P.ny;
    const int nf = DIR == 0 ? nx + 1 : ny + 1;
    const int nt = DIR == 0 ? ny : nx;
    const int A = DIR == 0 ? nt + 4 : nf, B = DIR == 0 ? nf : nt + 4;
    const int Bs = row_stride(B, ES);
    const int nfc = faces_computed(nf - 1, DIR == 0 ? P.bc[0] : P.bc[2]);
    const int bw = DIR == 0 ? nfc : nt; // extent of the lane index
    int tx, ty;
    tile_xy((bw + kGpX - 1) / kGpX, tx, ty);
    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int b = tx * kGpX + lane; // DIR 0: face, DIR 1: transverse cell
    const int a = ty * kGpY + w;    // DIR 0: transverse cell, DIR 1: face
    const int face = DIR == 0 ? b : a, tc = DIR == 0 ? a : b;
    // Lanes outside the grid take part in the staging and the barriers and
    // compute on whatever the slots hold there, but store nothing.
    const bool valid = face < nfc && tc < nt;
    const size_t AB = (size_t)A * Bs;
    // the host guarantees row_buffer_elems(nx, ny, DIR, 8) * 8 < 2^32 (the
    // FP32 buffer is half that size)
    const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)R, (short)0, (int)(unsigned)(row_buffer_elems(nx, ny, DIR, ES) * ES), 0x00020000);
    const unsigned plane = (unsigned)(AB * ES);
    const unsigned rstride = (unsigned)Bs * ES;
    // row r of the stencil = transverse index tc - 2 + r, stored at (tc + r);
    // the workgroup's first row starts at (ty kGpY, tx kGpX), 16-byte aligned
    const unsigned sbase = ((unsigned)(ty * kGpY) * (unsigned)Bs + (unsigned)(tx * kGpX)) * ES;
    using G = GpStage<DIR, T>;
    constexpr int L = kGpX / G::per16; // lanes per 64-element row segment
    const unsigned voff =
        DIR == 0 ? (unsigned)(lane % L) * 16u + (unsigned)(lane / L) * rstride : (unsigned)lane * 16u;
    RowReader<T> rv; // global reads for the positivity fallback
    rv.rsrc = rsrc;
    rv.plane = plane;
    {
        const unsigned a0 = DIR == 0 ? (unsigned)tc * Bs + face : (unsigned)face * Bs + tc;
        const unsigned bstride = DIR == 0 ? (unsigned)Bs : 1u;
#pragma unroll
        for (int r = 0; r < 5; ++r) rv.voff[r] = (a0 + r * bstride) * ES;
    }
    __shared__ T slot0[G::elems], slot1[G::elems], slot2[G::elems], slot3[G::elems];
    stage_component<DIR, T>(rsrc, slot0, sbase, plane, rstride, w, voff);
    stage_component<DIR, T>(rsrc, slot1, sbase + plane, plane, rstride, w, voff);
    stage_component<DIR, T>(rsrc, slot2, sbase + 2 * plane, plane, rstride, w, voff);
    stage_component<DIR, T>(rsrc, slot3, sbase + 3 * plane, plane, rstride, w, voff);
    const int lofs = w * G::len + lane;
    const StageReader<DIR, T> rd[4] = {{slot0 + lofs}, {slot1 + lofs}, {slot2 + lofs}, {slot3 + lofs}};
    const double ht = DIR == 0 ? P.dy : P.dx;
    const T iht = T(1.0 / ht);
    const double dt = S.dt;
    const PointPar par = point_par<2>(P.gamma, P.K, P.mu, dt);
    const T gam = T(par.gamma), Kt = T(par.K), iNt = T(par.iN);
    const bool weno = P.recon != 0;
    // Gauss sums of the outputs live in LDS (this lane's column), not in
    // registers across the Gauss-point loop: slot m = 4 q + k, q = 0 FL,
    // 1 FdL, 2 S0, 3 S1, 4 S2 (stage 2: FdL and S2 only, slots 0..7)
    constexpr int NQ = STAGE == 1 ? 5 : 2;
    __shared__ T sacc[NQ * 4][kGpX * kGpY];
    const int col = w * kGpX + lane;
    bool ok = valid;
#pragma unroll 1
    for (int g = 0; g < 3; ++g) {
        PointIn<T> in;
        T W0[4], Wl[4], Wr[4];
        // the first Gauss point waits for each component's copies in turn
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (g == 0) {
                if (k == 0) stage_wait<0>();
                else if (k == 1) stage_wait<1>();
                else if (k == 2) stage_wait<2>();
                else stage_wait<3>();
            }
            gp_noneq_k<T, T>(rd[k], g, k, iht, weno, in, Wl, Wr);
        }
        if (ok) {
            gp_fallback<T>(rv, weno, gam, Wl, Wr);
            NonEq<T, 2, T> ne;
            PointOut<T> o;
            ok = noneq_states<T, 2, T>(Wl, Wr, gam, Kt, iNt, ne, in.Wlx, in.Wly, in.Wrx, in.Wry);
            // the equilibrium inputs only now, so they are not held across
            // the non-equilibrium states
#pragma unroll
            for (int k = 0; k < 4; ++k) gp_equil_k<T, T>(rd[k], g, k, iht, in, W0);
            if (ok) {
                // equilibrium state: the kinetic average (WENO-Z) or the linear
                // value, selected per element so that every array stays in
                // registers
                T We[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) We[k] = weno ? ne.Xs[k] : W0[k];
                ok = gks_point<T, 2, T>(par, in, We, ne, o);
            }
            const T wg = g == 1 ? T(8.0 / 18.0) : T(5.0 / 18.0);
            if (ok) {
                const T* src[5] = {o.FL, o.FdL, o.S0, o.S1, o.S2};
#pragma unroll
                for (int q = 0; q < NQ; ++q)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const T v = wg * src[STAGE == 1 ? q : (q == 0 ? 1 : 4)][k];
                        T& sl = sacc[q * 4 + k][col];
                        sl = g == 0 ? v : sl + v;
                    }
            }
        }
    }
    if (!valid) return;
    if (!ok) {
        S.err = 1;
        return;
    }
    // Gauss sums into FP64; the MSMD face partials accumulate in FP64
    double acc[5][4];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[STAGE == 1 ? q : (q == 0 ? 1 : 4)][k] = double(sacc[q * 4 + k][col]);
    // back to the global frame
    const int gk[4] = {0, DIR == 0 ? 1 : 2, DIR == 0 ? 2 : 1, 3};
    const size_t nfa = DIR == 0 ? (size_t)ny * (nx + 1) : (size_t)(ny + 1) * nx;
    const size_t fi = DIR == 0 ? (size_t)tc * (nx + 1) + face : (size_t)face * nx + tc;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t o = (size_t)gk[k] * nfa + fi;
        if (STAGE == 1) {
            FL[o] = acc[0][k];
            FdL[o] = acc[1][k];
            Wfs[o] = msmd_half(acc[2][k], acc[3][k], acc[4][k], dt);
            Pf[o] = msmd_pred(acc[2][k], acc[3][k], acc[4][k], dt);
        } else {
            FdL[o] = acc[1][k];
            Wfs[o] = msmd_corr(Pf[o], acc[4][k], dt);
        }
    }
}

// 2-D cell update: one thread per cell.
template <int STAGE>
__global__ void __launch_bounds__(256) cell2d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS,
                                                     double* __restrict__ W, double* __restrict__ Wx,
                                                     double* __restrict__ Wy, double* __restrict__ PW,
                                                     const double* __restrict__ FLx, const double* __restrict__ FdLx,
                                                     const double* __restrict__ Wfx, const double* __restrict__ FLy,
                                                     const double* __restrict__ FdLy, const double* __restrict__ Wfy,
                                                     double* __restrict__ bmax)
{
    const ProbParam& P = PP[0];
    ProbState& S = PS[0];
    if (!S.active) return;
    const int nx = P.nx, ny = P.ny;
    int tx, ty;
    tile_xy((nx + blockDim.x - 1) / blockDim.x, tx, ty);
    const int i = tx * blockDim.x + threadIdx.x;
    const int j = ty * blockDim.y + threadIdx.y;
    const bool live = i < nx && j < ny;
    const int cur = S.cur, nxt = 1 - cur;
    const double dt = S.dt, idx = 1.0 / P.dx, idy = 1.0 / P.dy;
    const size_t plane = (size_t)nx * ny;
    const size_t nfx = (size_t)ny * (nx + 1), nfy = (size_t)(ny + 1) * nx;
    double wn[4];
    if (live) {
        const size_t c = (size_t)j * nx + i;
        const size_t fx = (size_t)j * (nx + 1) + i, fy = (size_t)j * nx + i;
        // right and top faces; a periodic direction's last face is its first
        const size_t fxr = (P.bc[0] == 0 && i == nx - 1) ? fx - i : fx + 1;
        const size_t fyt = (P.bc[2] == 0 && j == ny - 1) ? (size_t)i : fy + nx;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double dL = -(FdLx[k * nfx + fxr] - FdLx[k * nfx + fx]) * idx -
                              (FdLy[k * nfy + fyt] - FdLy[k * nfy + fy]) * idy;
            if (STAGE == 1) {
                const double L = -(FLx[k * nfx + fxr] - FLx[k * nfx + fx]) * idx -
                                 (FLy[k * nfy + fyt] - FLy[k * nfy + fy]) * idy;
                const double w = W[((size_t)cur * 4 + k) * plane + c];
                W[((size_t)nxt * 4 + k) * plane + c] = msmd_half(w, L, dL, dt);
                PW[k * plane + c] = msmd_pred(w, L, dL, dt);
            } else {
                wn[k] = msmd_corr(PW[k * plane + c], dL, dt);
                W[((size_t)nxt * 4 + k) * plane + c] = wn[k];
            }
            Wx[((size_t)nxt * 4 + k) * plane + c] = (Wfx[k * nfx + fxr] - Wfx[k * nfx + fx]) * idx;
            Wy[((size_t)nxt * 4 + k) * plane + c] = (Wfy[k * nfy + fyt] - Wfy[k * nfy + fy]) * idy;
        }
    }
    if (STAGE == 2) {
        double s = 0.0;
        if (live) {
            const double rho = wn[0], U = wn[1] / rho, V = wn[2] / rho;
            const double p = (P.gamma - 1.0) * (wn[3] - 0.5 * rho * (U * U + V * V));
            if (!(rho > 0.0) || !(p > 0.0)) S.err = 1;
            else {
                const double c = sqrt(P.gamma * p / rho);
                s = fmax((fabs(U) + c) * idx, (fabs(V) + c) * idy);
            }
        }
        // one plain store per workgroup; finish2d_kernel takes the maximum
        // (thousands of atomics on one address would queue at the memory side)
        const double m = block_max(s);
        if (threadIdx.x + threadIdx.y * blockDim.x == 0) bmax[blockIdx.x] = m;
    }
}

// Commit of a 2-D step (one workgroup): the largest signal speed over the
// second-stage cell-update workgroups' maxima bmax[0..nb), then the step as
// finish_kernel commits it.
__global__ void __launch_bounds__(256) finish2d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS,
                                                       const double* __restrict__ bmax, int nb)
{
    ProbState& S = PS[0];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v = fmax(v, bmax[b]);
    const double m = block_max(v);
    if (threadIdx.x == 0 && S.active) {
        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
        if (m > 0.0 && mb > S.smax) S.smax = mb;
        finish_problem(PP[0], S, 1, 2);
    }
}

__global__ void __launch_bounds__(256) signal2d_kernel(const ProbParam* __restrict__ PP, ProbState* __restrict__ PS,
                                                       const double* __restrict__ W)
{
    const ProbParam& P = PP[0];
    ProbState& S = PS[0];
    const int nx = P.nx, ny = P.ny;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const size_t plane = (size_t)nx * ny;
    double s = 0.0;
    if (i < nx && j < ny) {
        const size_t c = (size_t)j * nx + i;
        const double* Wb = W + (size_t)S.cur * 4 * plane;
        const double rho = Wb[c], U = Wb[plane + c] / rho, V = Wb[2 * plane + c] / rho;
        const double p = (P.gamma - 1.0) * (Wb[3 * plane + c] - 0.5 * rho * (U * U + V * V));
        if (!(rho > 0.0) || !(p > 0.0)) S.err = 1;
        else {
            const double cs = sqrt(P.gamma * p / rho);
            s = fmax((fabs(U) + cs) * (1.0 / P.dx), (fabs(V) + cs) * (1.0 / P.dy)); // as in the step kernels
        }
    }
    block_max_atomic(s, &S.smax);
}

} // namespace gks
