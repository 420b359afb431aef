// gks_api.hip -- host side of the C ABI declared in include/gks.h.
#include "../../include/gks.h"
#include "gks_kernels.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>
#include <mutex>

using gks::ProbParam;
using gks::ProbState;
using gks::Tile;

namespace {

thread_local std::string g_init_error;

struct EventPair {
    hipEvent_t a, b;
    int kind;
};

} // namespace

struct gks_handle {
    int dim = 0, nprob = 0, precision = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<ProbParam> hp;
    ProbParam* dP = nullptr;
    ProbState* dS = nullptr;
    long long Ntot = 0, F = 0; // 1-D cells and faces
    Tile* dTilesC = nullptr; // 1-D cell tiles of kBlock1D (signal-speed kernel)
    int nTilesC = 0;
    double *W = nullptr, *Wx = nullptr, *Wy = nullptr, *PW = nullptr;
    double *FL = nullptr, *FdL = nullptr, *Wfs = nullptr, *Pf = nullptr;
    double *FLy = nullptr, *FdLy = nullptr, *Wfsy = nullptr, *Pfy = nullptr;
    double* bmax = nullptr; // 2-D: per-workgroup signal-speed maxima of the cell update
    int nbmax = 0;
    void *Rx = nullptr, *Ry = nullptr; // face-row buffers: double (FP64) or float (FP32-mixed)
    double* R1 = nullptr; // 1-D two-kernel steps: reconstructed faces
    double* stage = nullptr; // transpose staging
    size_t stage_len = 0;
    std::string err;
    bool dead = false; // a HIP call failed: the device state is not trusted any more
    bool timing = false;
    std::vector<EventPair> pending;
    std::vector<EventPair> pool;
    double tot_ms[3] = {0, 0, 0};
    long long launches[3] = {0, 0, 0};
    long long last_updates = 0;
    // batched 1-D: work items per tile size, device work counters
    unsigned* ctr = nullptr;
    Tile* dItems[3] = {nullptr, nullptr, nullptr}; // tile sizes 64, 128, 256 (BLK - 1 cells each)
    int nItems[3] = {0, 0, 0};
    int* dFirst[3] = {nullptr, nullptr, nullptr}; // per problem: first item and item count
    int* dCount[3] = {nullptr, nullptr, nullptr};
    Tile* dAct[3] = {nullptr, nullptr, nullptr};  // items of the active problems (rebuilt every step)
    int* dNact = nullptr;
    int act_list = -1; // item list (index) the device work list was last built from (-1: stale)
    std::vector<int> hcount[3]; // per problem: items of each tile size (host copy)
    std::vector<char> last_active; // problem still running after the last gks_step (host copy)
    // lane-pair steps: while the active work items of the tuned tile size
    // are at most half the CUs, the steps run the 256-thread kernel whose lane
    // pairs share a face, on tiles of 127 cells (GKS_SPLIT: 0 never,
    // 1 automatic (default), 2 always)
    int split = 0, split_mode = 1;
    // two-kernel steps: while the active 255-cell work items are at least
    // kPhaseItemsPerCU per CU, each stage runs as the face kernel and the
    // point-and-cell kernel (GKS_PHASES: 0 never, 1 automatic (default),
    // 2 always)
    int phases = 0, phases_mode = 1;
    int ncu = 256;
    // launch configuration (autotuned): threads per tile, workgroups per CU
    // (0: one workgroup per work item)
    bool tuned = false;
    int blk = 128, gmul = 2;
    std::string tune_note, cfg_text;
    ProbState last_state{}; // problem state read by the last gks_state call
    // step graph
    bool use_graph = true;
    hipStream_t cap = nullptr;
    // 2-D: the y-face kernels run on a second stream, forked from and joined
    // to the step's stream around them (not while kernels are being timed)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // graphs of 1, kGraphSteps[0] and kGraphSteps[1] steps
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
};

namespace {

int fail(gks_handle* h, int code, const std::string& msg)
{
    if (h) h->err = msg;
    else g_init_error = msg;
    return code;
}

// a HIP runtime failure on a handle leaves it unusable (GKS_ESTATE from then on)
int fail_hip(gks_handle* h, hipError_t e, const char* what)
{
    if (h) h->dead = true;
    return fail(h, e == hipErrorOutOfMemory ? GKS_ENOMEM : GKS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int dead_handle(gks_handle* h)
{
    return fail(h, GKS_ESTATE, "handle unusable after an earlier HIP runtime error (" + h->err + ")");
}

#define HIP_TRY(h, expr)                                                                          \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail_hip(h, e_, #expr);                                      \
    } while (0)

template <typename Ptr> hipError_t dalloc(Ptr** p, size_t n)
{
    return hipMalloc((void**)p, n * sizeof(Ptr));
}

void dfree(void* p)
{
    if (p) (void)hipFree(p);
}

// AoS [cells][nv] (with ld = nv) <-> SoA [nv][cells], nv = 3 or 4.  For
// 1-D the SoA slots are (rho, rho U, rho E).
__global__ void aos_to_soa(const double* __restrict__ src, double* __restrict__ dst, long long n, int nv, long long ld)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int k = 0; k < nv; ++k) dst[k * ld + c] = src[c * nv + k];
}
__global__ void soa_to_aos(const double* __restrict__ src, double* __restrict__ dst, long long n, int nv, long long ld)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int k = 0; k < nv; ++k) dst[c * nv + k] = src[k * ld + c];
}

int validate(const gks_problem* pr, int32_t nprob, int32_t precision)
{
    if (!pr || nprob < 1) return fail(nullptr, GKS_EINVAL, "no problems given");
    if (precision != GKS_PREC_FP64 && precision != GKS_PREC_FP32_MIXED)
        return fail(nullptr, GKS_EINVAL, "unknown precision");
    const int dim = pr[0].dim;
    if (dim != 1 && dim != 2) return fail(nullptr, GKS_EINVAL, "dim must be 1 or 2");
    if (dim == 2 && nprob != 1) return fail(nullptr, GKS_EINVAL, "a 2-D handle holds exactly one problem");
    for (int p = 0; p < nprob; ++p) {
        const gks_problem& q = pr[p];
        char buf[160];
        auto bad = [&](const char* what) {
            snprintf(buf, sizeof buf, "problem %d: %s", p, what);
            return fail(nullptr, GKS_EINVAL, buf);
        };
        if (q.dim != dim) return bad("all problems of a handle must have the same dim");
        if (q.nx < 4 || (dim == 2 && q.ny < 4) || (dim == 1 && q.ny != 1 && q.ny != 0)) return bad("bad nx/ny");
        if ((long long)q.nx * (dim == 2 ? q.ny : 1) > (1ll << 31) - 1) return bad("too many cells");
        // 2-D face-row buffers are read through 32-bit byte offsets
        if (dim == 2 && std::max(gks::row_buffer_elems(q.nx, q.ny, 0), gks::row_buffer_elems(q.nx, q.ny, 1)) * 8 >
                            0xffffffffll)
            return bad("2-D grid too large for one handle (at most about 4370 x 4370 cells)");
        if (!(q.xhi > q.xlo) || (dim == 2 && !(q.yhi > q.ylo))) return bad("empty domain");
        if (!(q.gamma > 1.0) || !std::isfinite(q.gamma)) return bad("gamma must be > 1");
        if (!(q.mu >= 0.0) || !std::isfinite(q.mu)) return bad("mu must be >= 0");
        if (!(q.dt_fixed > 0.0) && !(q.cfl > 0.0)) return bad("need cfl > 0 or dt_fixed > 0");
        if (!(q.t_end > 0.0)) return bad("t_end must be > 0");
        if (q.order != 6 && q.order != 8) return bad("order must be 6 or 8");
        if (q.recon != GKS_RECON_LINEAR && q.recon != GKS_RECON_WENOZ) return bad("unknown recon");
        const int nb = dim == 2 ? 4 : 2;
        for (int k = 0; k < nb; ++k) {
            const int b = q.bc[k];
            if (b < GKS_BC_PERIODIC || b > GKS_BC_CHAR) return bad("unknown boundary condition");
            if (b == GKS_BC_SPLIT && dim != 2) return bad("split boundaries are 2-D only");
            if (b == GKS_BC_CHAR && dim != 1) return bad("characteristic boundaries are 1-D only");
            if (b == GKS_BC_SPLIT && q.bc_beyond[k] != GKS_BC_REFLECT && q.bc_beyond[k] != GKS_BC_INFLOW)
                return bad("bc_beyond of a split side must be GKS_BC_REFLECT or GKS_BC_INFLOW");
            if (b == GKS_BC_SPLIT && !(std::isfinite(q.bc_split[k][0]) && std::isfinite(q.bc_split[k][1])))
                return bad("bc_split must be finite");
            // the states a side uses must be physical
            const int nst = b == GKS_BC_INFLOW ? 1 : (b == GKS_BC_SPLIT ? (q.bc_beyond[k] == GKS_BC_INFLOW ? 2 : 1) : 0);
            for (int a = 0; a < nst; ++a) {
                const double* st = q.bc_state[k][a];
                const double rho = st[0], U = st[1] / rho, V = dim == 2 ? st[2] / rho : 0.0;
                const double pr = (q.gamma - 1.0) * (st[3] - 0.5 * rho * (U * U + V * V));
                if (!(rho > 0.0) || !(pr > 0.0) || !std::isfinite(pr)) return bad("non-physical boundary state");
            }
        }
        for (int k = 0; k < nb; k += 2)
            if ((q.bc[k] == GKS_BC_PERIODIC) != (q.bc[k + 1] == GKS_BC_PERIODIC))
                return bad("periodic boundaries must be paired");
    }
    return GKS_OK;
}

void record(gks_handle* h, hipStream_t st, int kind, bool begin)
{
    if (!h->timing || st != h->stream) return;
    if (begin) {
        EventPair e;
        if (!h->pool.empty()) {
            e = h->pool.back();
            h->pool.pop_back();
        } else {
            (void)hipEventCreate(&e.a);
            (void)hipEventCreate(&e.b);
        }
        e.kind = kind;
        (void)hipEventRecord(e.a, h->stream);
        h->pending.push_back(e);
    } else {
        (void)hipEventRecord(h->pending.back().b, h->stream);
    }
}

void harvest(gks_handle* h)
{
    for (auto& e : h->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            h->tot_ms[e.kind] += ms;
            h->launches[e.kind] += 1;
        }
        h->pool.push_back(e);
    }
    h->pending.clear();
}

// the device work list for the current tile size, rebuilt from the problem
// states when it is stale (first step, tile size changed, state restored)
// item list of the current launch shape: the tuned tile size, or the
// 127-cell tiles of the lane-pair kernel
int list_index(const gks_handle* h)
{
    return h->split ? 1 : (h->phases ? 2 : (h->blk == 64 ? 0 : (h->blk == 128 ? 1 : 2)));
}

void ensure_work_list(gks_handle* h, hipStream_t st)
{
    const int b = list_index(h);
    if (h->act_list == b) return;
    gks::compact_items_kernel<<<1, gks::kCompactThreads, 0, st>>>(h->dS, h->nprob, h->dItems[b], h->dFirst[b],
                                                                  h->dCount[b], h->dAct[b], h->dNact);
    h->act_list = b;
}

template <typename T> void launch_step_1d(gks_handle* h, hipStream_t st)
{
    const int b = list_index(h);
    const int n = h->nItems[b];
    ensure_work_list(h, st);
    Tile* it = h->dAct[b];
    int* na = h->dNact;
    const int G = h->gmul == 0 ? n : std::min(n, h->gmul * h->ncu);
    record(h, st, 0, true);
    if (h->phases) {
        // one workgroup per item of the full list; R1 holds T values
        double* W = h->W;
        double* X = h->Wx;
        T* R1 = reinterpret_cast<T*>(h->R1);
        gks::face1d_kernel<T, 1><<<n, gks::kPhaseBlk, 0, st>>>(h->dP, h->dS, it, na, W, X, R1, h->Ntot, h->F);
        gks::pointcell1d_kernel<T, 1><<<n, gks::kPhaseBlk, 0, st>>>(h->dP, h->dS, it, na, R1, W, X, h->PW, h->Pf, h->Ntot, h->F);
        gks::face1d_kernel<T, 2><<<n, gks::kPhaseBlk, 0, st>>>(h->dP, h->dS, it, na, W, X, R1, h->Ntot, h->F);
        gks::pointcell1d_kernel<T, 2><<<n, gks::kPhaseBlk, 0, st>>>(h->dP, h->dS, it, na, R1, W, X, h->PW, h->Pf, h->Ntot, h->F);
    } else if (h->split) {
        const int Gs = std::min(n, std::max(1, h->gmul) * h->ncu);
        gks::stage1d_kernel<T, 1, 256, 2><<<Gs, 256, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->W, h->Wx, h->PW, h->Pf, h->Ntot, h->F);
        gks::stage1d_kernel<T, 2, 256, 2><<<Gs, 256, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->W, h->Wx, h->PW, h->Pf, h->Ntot, h->F);
    } else if (h->blk == 64) {
        gks::stage1d_kernel<T, 1, 64><<<G, 64, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->W, h->Wx, h->PW, h->Pf, h->Ntot, h->F);
        gks::stage1d_kernel<T, 2, 64><<<G, 64, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->W, h->Wx, h->PW, h->Pf, h->Ntot, h->F);
    } else if (h->blk == 128) {
        gks::stage1d_kernel<T, 1, 128><<<G, 128, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->W, h->Wx, h->PW, h->Pf, h->Ntot, h->F);
        gks::stage1d_kernel<T, 2, 128><<<G, 128, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->W, h->Wx, h->PW, h->Pf, h->Ntot, h->F);
    } else {
        gks::stage1d_kernel<T, 1, 256><<<G, 256, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->W, h->Wx, h->PW, h->Pf, h->Ntot, h->F);
        gks::stage1d_kernel<T, 2, 256><<<G, 256, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->W, h->Wx, h->PW, h->Pf, h->Ntot, h->F);
    }
    // the step's commit (and the work list's rebuild when a problem has
    // stopped) in a one-workgroup launch
    gks::commit1d_kernel<<<1, gks::kPhaseBlk, 0, st>>>(h->dP, h->dS, it, na, h->ctr, h->nprob, h->dItems[b], h->dFirst[b], h->dCount[b]);
    record(h, st, 0, false);
    h->act_list = b;
}

// workgroups of the 2-D cell update: tiles of 64 x 4 cells
int cell_blocks(int nx, int ny) { return ((nx + 63) / 64) * ((ny + 3) / 4); }

template <typename T> void launch_step_2d(gks_handle* h, hipStream_t st)
{
    const ProbParam& P = h->hp[0];
    const int nx = P.nx, ny = P.ny;
    const dim3 br(64, 4), bg(gks::kGpX, gks::kGpY), bc(64, 4);
    // 1-D grids of 2-D tiles; the kernels map workgroups to tiles per XCD.
    // x faces: rows (ny + 4) x faces (nx + 1); y faces: faces (ny + 1) x columns (nx + 4)
    auto tiles = [](int ext_x, int ext_y, dim3 b) { return ((ext_x + b.x - 1) / b.x) * ((ext_y + b.y - 1) / b.y); };
    const int grx = tiles(gks::faces_computed(nx, P.bc[0]), ny + 4, br), gry = tiles(nx + 4, gks::faces_computed(ny, P.bc[2]), br);
    const int ggx = tiles(gks::faces_computed(nx, P.bc[0]), ny, bg), ggy = tiles(nx, gks::faces_computed(ny, P.bc[2]), bg);
    const int gc = tiles(nx, ny, bc); // == cell_blocks(nx, ny) == h->nbmax
    // The x-face and y-face kernels of a stage are independent until the cell
    // update: the y-face pair runs on the side stream, so that the two chains
    // overlap (each fills the other's partly idle last wave of workgroups).
    // Kernel timing keeps every launch on the handle's stream.
    const bool fork = h->side && !h->timing;
    hipStream_t sy = fork ? h->side : st;
    for (int stage = 1; stage <= 2; ++stage) {
        if (fork) {
            (void)hipEventRecord(h->ev_fork, st);
            (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
        }
        record(h, st, 1, true);
        if (P.order == 8)
            gks::row2d_kernel<T, 0, 8><<<grx, br, 0, st>>>(h->dP, h->dS, h->W, h->Wx, h->Wy, stage, (T*)h->Rx);
        else
            gks::row2d_kernel<T, 0, 6><<<grx, br, 0, st>>>(h->dP, h->dS, h->W, h->Wx, h->Wy, stage, (T*)h->Rx);
        record(h, st, 1, false);
        record(h, st, 0, true);
        if (stage == 1)
            gks::gp2d_kernel<T, 0, 1><<<ggx, bg, 0, st>>>(h->dP, h->dS, (const T*)h->Rx, h->FL, h->FdL, h->Wfs, h->Pf);
        else
            gks::gp2d_kernel<T, 0, 2><<<ggx, bg, 0, st>>>(h->dP, h->dS, (const T*)h->Rx, h->FL, h->FdL, h->Wfs, h->Pf);
        record(h, st, 0, false);
        record(h, sy, 1, true);
        if (P.order == 8)
            gks::row2d_kernel<T, 1, 8><<<gry, br, 0, sy>>>(h->dP, h->dS, h->W, h->Wx, h->Wy, stage, (T*)h->Ry);
        else
            gks::row2d_kernel<T, 1, 6><<<gry, br, 0, sy>>>(h->dP, h->dS, h->W, h->Wx, h->Wy, stage, (T*)h->Ry);
        record(h, sy, 1, false);
        record(h, sy, 0, true);
        if (stage == 1)
            gks::gp2d_kernel<T, 1, 1><<<ggy, bg, 0, sy>>>(h->dP, h->dS, (const T*)h->Ry, h->FLy, h->FdLy, h->Wfsy, h->Pfy);
        else
            gks::gp2d_kernel<T, 1, 2><<<ggy, bg, 0, sy>>>(h->dP, h->dS, (const T*)h->Ry, h->FLy, h->FdLy, h->Wfsy, h->Pfy);
        record(h, sy, 0, false);
        if (fork) {
            (void)hipEventRecord(h->ev_join, h->side);
            (void)hipStreamWaitEvent(st, h->ev_join, 0);
        }
        record(h, st, 2, true);
        if (stage == 1)
            gks::cell2d_kernel<1><<<gc, bc, 0, st>>>(h->dP, h->dS, h->W, h->Wx, h->Wy, h->PW, h->FL, h->FdL, h->Wfs,
                                                      h->FLy, h->FdLy, h->Wfsy, h->bmax);
        else
            gks::cell2d_kernel<2><<<gc, bc, 0, st>>>(h->dP, h->dS, h->W, h->Wx, h->Wy, h->PW, h->FL, h->FdL, h->Wfs,
                                                      h->FLy, h->FdLy, h->Wfsy, h->bmax);
        record(h, st, 2, false);
    }
    gks::finish2d_kernel<<<1, 256, 0, st>>>(h->dP, h->dS, h->bmax, gc);
}

void launch_step(gks_handle* h, hipStream_t st)
{
    if (h->dim == 1) {
        if (h->precision == GKS_PREC_FP64) launch_step_1d<double>(h, st);
        else launch_step_1d<float>(h, st);
    } else {
        if (h->precision == GKS_PREC_FP64) launch_step_2d<double>(h, st);
        else launch_step_2d<float>(h, st);
    }
}

void drop_graph(gks_handle* h)
{
    for (int g = 0; g < 3; ++g) {
        if (h->gexec[g]) (void)hipGraphExecDestroy(h->gexec[g]);
        if (h->graph[g]) (void)hipGraphDestroy(h->graph[g]);
        h->gexec[g] = nullptr;
        h->graph[g] = nullptr;
    }
}

// two-kernel steps while the active 255-cell work items number at least
// this many per CU (1 to 4 measured within 1 % of each other on the
// 256-problem batch)
constexpr int kPhaseItemsPerCU = 2;

// steps per replay of the longer graphs: fewer graph launches, so fewer
// gaps between steps (about 8 us each) and less host work per step
constexpr int kGraphSteps[2] = {8, 32};

// capture one MSMD step, and kGraphSteps[g] steps in a row, (kernel nodes
// only) on the private capture stream; a step's launches depend only on
// device state, so a replay of a long graph equals as many replays of the
// short one
int build_graph(gks_handle* h)
{
    drop_graph(h);
    if (h->dim == 1) ensure_work_list(h, h->stream); // the captured step assumes a current list
    for (int g = 0; g < 3; ++g) {
        const int n = g == 0 ? 1 : kGraphSteps[g - 1];
        HIP_TRY(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        for (int s = 0; s < n; ++s) launch_step(h, h->cap);
        HIP_TRY(h, hipStreamEndCapture(h->cap, &h->graph[g]));
        HIP_TRY(h, hipGraphInstantiate(&h->gexec[g], h->graph[g], nullptr, nullptr, 0));
    }
    return GKS_OK;
}

// ---------------------------------------------------------------------------
// Autotuner for the batched 1-D path: tile size (64, 128, 256 threads) and
// grid size (1, 2, 4 persistent workgroups per CU, or one workgroup per work
// item); each candidate runs 1 + 2 steps (the last two timed) from the same
// saved state, which is restored afterwards.  All candidates run the same
// per-face and per-cell arithmetic, so the choice does not change results.
// GKS_TUNE="BLK:GMUL" forces a configuration; GKS_TUNE_CACHE names a text
// file of "signature blk gmul" lines read before and appended after tuning.
// ---------------------------------------------------------------------------
std::string tune_signature(const gks_handle* h)
{
    int maxnx = 0;
    for (const auto& P : h->hp) maxnx = std::max(maxnx, P.nx);
    char buf[160];
    snprintf(buf, sizeof buf, "dim1:np%d:N%lld:max%d:prec%d:cu%d", h->nprob, h->Ntot, maxnx, h->precision, h->ncu);
    return buf;
}

bool parse_forced(const char* s, int& blk, int& gmul)
{
    int b = 0, g = -1;
    char tail = 0;
    if (sscanf(s, "%d:%d%c", &b, &g, &tail) == 2 && (b == 64 || b == 128 || b == 256) && g >= 0 && g <= 16) {
        blk = b;
        gmul = g;
        return true;
    }
    return false;
}

int autotune(gks_handle* h)
{
    h->tuned = true;
    if (const char* f = getenv("GKS_TUNE")) {
        if (!parse_forced(f, h->blk, h->gmul)) {
            h->tuned = false;
            return fail(h, GKS_EINVAL, std::string("bad GKS_TUNE (want BLK:GMUL, BLK 64/128/256, GMUL 0..16): ") + f);
        }
        h->tune_note = std::string("forced ") + f;
        return GKS_OK;
    }
    const std::string sig = tune_signature(h);
    const char* cache = getenv("GKS_TUNE_CACHE");
    if (cache) {
        if (FILE* fp = fopen(cache, "r")) {
            char line[256];
            while (fgets(line, sizeof line, fp)) {
                char key[200];
                int b, g;
                if (sscanf(line, "%199s %d %d", key, &b, &g) == 3 && sig == key && (b == 64 || b == 128 || b == 256) &&
                    g >= 0 && g <= 16) {
                    h->blk = b; h->gmul = g;
                    h->tune_note = "cache " + sig;
                }
            }
            fclose(fp);
            if (!h->tune_note.empty()) return GKS_OK;
        }
    }
    // save state (all three slots) and bookkeeping
    const size_t nW = (size_t)3 * 3 * h->Ntot;
    double *sW = nullptr, *sX = nullptr;
    std::vector<ProbState> s0(h->nprob);
    HIP_TRY(h, dalloc(&sW, nW));
    HIP_TRY(h, dalloc(&sX, nW));
    HIP_TRY(h, hipMemcpyAsync(sW, h->W, nW * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(sX, h->Wx, nW * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(s0.data(), h->dS, sizeof(ProbState) * h->nprob, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    // Candidates from larger tiles and fewer workgroups to smaller and more;
    // a later one is taken only when it is more than 3 % faster.  The two
    // timed steps run with every problem active, but a run's later steps
    // hold fewer items than workgroups, where each launch costs more with
    // more, smaller workgroups (256-thread tiles on one workgroup per CU
    // and 128-thread tiles on two time alike at full load, yet the second
    // takes 8 % longer over the whole 256-problem run).
    struct Cand { int blk, gmul; };
    std::vector<Cand> cands;
    for (int b : {256, 128, 64})
        for (int g : {1, 2, 4, 0}) cands.push_back({b, g});
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    float best = 1e30f;
    Cand bc = cands[0];
    const bool was_timing = h->timing;
    h->timing = false;
    int st = GKS_OK;
    for (const Cand& c : cands) {
        h->blk = c.blk; h->gmul = c.gmul;
        launch_step(h, h->stream);
        (void)hipEventRecord(e0, h->stream);
        launch_step(h, h->stream);
        launch_step(h, h->stream);
        (void)hipEventRecord(e1, h->stream);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = fail(h, GKS_EDEVICE, "autotune: timing failed");
            break;
        }
        if (ms < 0.97f * best) { best = ms; bc = c; }
        // restore
        if (hipMemcpyAsync(h->W, sW, nW * sizeof(double), hipMemcpyDeviceToDevice, h->stream) != hipSuccess ||
            hipMemcpyAsync(h->Wx, sX, nW * sizeof(double), hipMemcpyDeviceToDevice, h->stream) != hipSuccess ||
            hipMemcpyAsync(h->dS, s0.data(), sizeof(ProbState) * h->nprob, hipMemcpyHostToDevice, h->stream) !=
                hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess) {
            st = fail(h, GKS_EDEVICE, "autotune: state restore failed");
            break;
        }
        h->act_list = -1; // the work list reflects the tuning steps, not the restored state
    }
    h->act_list = -1;
    h->timing = was_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dfree(sW);
    dfree(sX);
    if (st) return st;
    h->blk = bc.blk; h->gmul = bc.gmul;
    char note[200];
    snprintf(note, sizeof note, "tuned %s: blk %d gmul %d (%.3f ms for 2 steps)", sig.c_str(), bc.blk, bc.gmul, best);
    h->tune_note = note;
    if (cache) {
        if (FILE* fp = fopen(cache, "a")) {
            fprintf(fp, "%s %d %d\n", sig.c_str(), bc.blk, bc.gmul);
            fclose(fp);
        }
    }
    return GKS_OK;
}

void release(gks_handle* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void* p : {(void*)h->dP, (void*)h->dS, (void*)h->dTilesC, (void*)h->W, (void*)h->Wx,
                    (void*)h->Wy, (void*)h->PW, (void*)h->FL, (void*)h->FdL, (void*)h->Wfs, (void*)h->Pf,
                    (void*)h->FLy, (void*)h->FdLy, (void*)h->Wfsy, (void*)h->Pfy, (void*)h->Rx, (void*)h->Ry,
                    (void*)h->R1, (void*)h->stage, (void*)h->bmax})
        dfree(p);
    drop_graph(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    dfree(h->ctr);
    for (int b = 0; b < 3; ++b) {
        dfree(h->dItems[b]);
        dfree(h->dFirst[b]);
        dfree(h->dCount[b]);
        dfree(h->dAct[b]);
    }
    dfree(h->dNact);
    for (auto& e : h->pending) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (auto& e : h->pool) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

// Device-side parameters of one problem (cells from coff, faces from foff
// in the batched 1-D arrays).
ProbParam make_param(const gks_problem& q, int dim, long long coff, long long foff)
{
    ProbParam P{};
    P.nx = q.nx;
    P.ny = dim == 2 ? q.ny : 1;
    P.coff = coff;
    P.foff = foff;
    P.dx = (q.xhi - q.xlo) / q.nx;
    P.dy = dim == 2 ? (q.yhi - q.ylo) / q.ny : 1.0;
    P.gamma = q.gamma;
    P.K = dim == 1 ? (3.0 - q.gamma) / (q.gamma - 1.0) : (4.0 - 2.0 * q.gamma) / (q.gamma - 1.0);
    P.mu = q.mu;
    P.cfl = q.cfl;
    P.dt_fixed = q.dt_fixed;
    P.t_end = q.t_end;
    P.order = q.order;
    P.recon = q.recon;
    for (int k = 0; k < 4; ++k) P.bc[k] = (dim == 1 && k >= 2) ? 0 : q.bc[k];
    P.xlo = q.xlo;
    P.ylo = dim == 2 ? q.ylo : 0.0;
    for (int k = 0; k < 4; ++k) {
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 4; ++c) P.bstate[k][a][c] = q.bc_state[k][a][c];
        P.bsplit[k][0] = q.bc_split[k][0];
        P.bsplit[k][1] = q.bc_split[k][1];
        P.bbeyond[k] = q.bc_beyond[k];
    }
    return P;
}

int init_common(const gks_problem* probs, int32_t nprob, int32_t precision, const double* const* W0,
                const double* const* Wx0, const double* const* Wy0, void* stream, gks_handle** out, bool device)
{
    if (!out) return fail(nullptr, GKS_EINVAL, "out is NULL");
    *out = nullptr;
    int st = validate(probs, nprob, precision);
    if (st) return st;
    const int dim = probs[0].dim;
    for (int p = 0; p < nprob; ++p)
        if (!W0 || !Wx0 || !W0[p] || !Wx0[p] || (dim == 2 && (!Wy0 || !Wy0[p])))
            return fail(nullptr, GKS_EINVAL, "missing initial data array");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(nullptr, GKS_EDEVICE, "no HIP device available");

    gks_handle* h = new gks_handle();
    h->dim = dim;
    h->nprob = nprob;
    h->precision = precision;
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreate(&h->stream) != hipSuccess) {
            delete h;
            return fail(nullptr, GKS_EDEVICE, "hipStreamCreate failed");
        }
        h->own_stream = true;
    }
    auto bail = [&](int code) {
        g_init_error = h->err;
        release(h);
        return code;
    };
#define TRY(expr)                                                                                 \
    do {                                                                                          \
        int s_ = (expr);                                                                          \
        if (s_) return bail(s_);                                                                  \
    } while (0)

    // problem parameters, tiles
    std::vector<Tile> tc;
    long long coff = 0, foff = 0;
    for (int p = 0; p < nprob; ++p) {
        const gks_problem& q = probs[p];
        const ProbParam P = make_param(q, dim, coff, foff);
        h->hp.push_back(P);
        if (dim == 1) {
            for (int s = 0; s < q.nx; s += gks::kBlock1D) tc.push_back(Tile{p, s});
            coff += q.nx;
            foff += q.nx + 1;
        }
    }
    h->Ntot = dim == 1 ? coff : (long long)probs[0].nx * probs[0].ny;
    h->F = foff;
    const int nv = dim + 2;
    TRY(([&]() -> int { HIP_TRY(h, dalloc(&h->dP, nprob)); HIP_TRY(h, dalloc(&h->dS, nprob)); return 0; })());
    TRY(([&]() -> int {
        HIP_TRY(h, hipMemcpyAsync(h->dP, h->hp.data(), sizeof(ProbParam) * nprob, hipMemcpyHostToDevice, h->stream));
        std::vector<ProbState> s0(nprob);
        for (auto& s : s0) { s = ProbState{}; s.active = 1; }
        HIP_TRY(h, hipMemcpyAsync(h->dS, s0.data(), sizeof(ProbState) * nprob, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        return 0;
    })());
    const long long N = h->Ntot;
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            h->ncu = ncu;
    }
    if (const char* g = getenv("GKS_GRAPH")) h->use_graph = atoi(g) != 0;
    if (const char* g = getenv("GKS_SPLIT")) h->split_mode = std::min(std::max(atoi(g), 0), 2);
    if (const char* g = getenv("GKS_PHASES")) h->phases_mode = std::min(std::max(atoi(g), 0), 2);
    if (dim != 1) h->phases_mode = 0;
    h->last_active.assign(nprob, 1);
    TRY(([&]() -> int {
        HIP_TRY(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        if (dim == 2) {
            HIP_TRY(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
            HIP_TRY(h, hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
            HIP_TRY(h, hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
        }
        HIP_TRY(h, dalloc(&h->ctr, 3));
        HIP_TRY(h, dalloc(&h->dNact, 1));
        HIP_TRY(h, hipMemset(h->ctr, 0, 3 * sizeof(unsigned)));
        return 0;
    })());
    if (dim == 1) {
        const int blks[3] = {64, 128, 256};
        for (int b = 0; b < 3; ++b) {
            std::vector<Tile> items;
            std::vector<int> first(nprob), count(nprob);
            for (int p = 0; p < nprob; ++p) {
                first[p] = (int)items.size();
                for (int s = 0; s < probs[p].nx; s += blks[b] - 1) items.push_back(Tile{p, s});
                count[p] = (int)items.size() - first[p];
            }
            h->nItems[b] = (int)items.size();
            h->hcount[b] = count;
            TRY(([&]() -> int {
                HIP_TRY(h, dalloc(&h->dItems[b], items.size()));
                HIP_TRY(h, dalloc(&h->dAct[b], items.size()));
                HIP_TRY(h, dalloc(&h->dFirst[b], (size_t)nprob));
                HIP_TRY(h, dalloc(&h->dCount[b], (size_t)nprob));
                HIP_TRY(h, hipMemcpy(h->dItems[b], items.data(), sizeof(Tile) * items.size(), hipMemcpyHostToDevice));
                HIP_TRY(h, hipMemcpy(h->dFirst[b], first.data(), sizeof(int) * nprob, hipMemcpyHostToDevice));
                HIP_TRY(h, hipMemcpy(h->dCount[b], count.data(), sizeof(int) * nprob, hipMemcpyHostToDevice));
                return 0;
            })());
        }
    } else {
        h->tuned = true;
    }
    if (dim == 1) {
        h->nTilesC = (int)tc.size();
        TRY(([&]() -> int {
            HIP_TRY(h, dalloc(&h->dTilesC, tc.size()));
            HIP_TRY(h, hipMemcpy(h->dTilesC, tc.data(), sizeof(Tile) * tc.size(), hipMemcpyHostToDevice));
            // three state slots: W^n, W^{n+1/2}, W^{n+1} (the batched stage
            // kernel never writes a slot that another item reads in the same launch)
            HIP_TRY(h, dalloc(&h->W, 3 * 3 * N));
            HIP_TRY(h, dalloc(&h->Wx, 3 * 3 * N));
            HIP_TRY(h, dalloc(&h->PW, 3 * N));
            HIP_TRY(h, dalloc(&h->Pf, 3 * h->F));
            return 0;
        })());
    } else {
        const long long nx = probs[0].nx, ny = probs[0].ny;
        TRY(([&]() -> int {
            HIP_TRY(h, dalloc(&h->W, 2 * 4 * N));
            HIP_TRY(h, dalloc(&h->Wx, 2 * 4 * N));
            HIP_TRY(h, dalloc(&h->Wy, 2 * 4 * N));
            HIP_TRY(h, dalloc(&h->PW, 4 * N));
            const long long nfx = ny * (nx + 1), nfy = (ny + 1) * nx;
            HIP_TRY(h, dalloc(&h->FL, 4 * nfx));
            HIP_TRY(h, dalloc(&h->FdL, 4 * nfx));
            HIP_TRY(h, dalloc(&h->Wfs, 4 * nfx));
            HIP_TRY(h, dalloc(&h->Pf, 4 * nfx));
            HIP_TRY(h, dalloc(&h->FLy, 4 * nfy));
            HIP_TRY(h, dalloc(&h->FdLy, 4 * nfy));
            HIP_TRY(h, dalloc(&h->Wfsy, 4 * nfy));
            HIP_TRY(h, dalloc(&h->Pfy, 4 * nfy));
            h->nbmax = cell_blocks((int)nx, (int)ny);
            HIP_TRY(h, dalloc(&h->bmax, h->nbmax));
            const int es = precision == GKS_PREC_FP64 ? 8 : 4;
            HIP_TRY(h, hipMalloc(&h->Rx, (size_t)gks::row_buffer_elems((int)nx, (int)ny, 0, es) * es));
            HIP_TRY(h, hipMalloc(&h->Ry, (size_t)gks::row_buffer_elems((int)nx, (int)ny, 1, es) * es));
            return 0;
        })());
    }
    // upload: AoS -> SoA through a staging buffer
    long long maxcells = 0;
    for (int p = 0; p < nprob; ++p) maxcells = std::max<long long>(maxcells, (long long)h->hp[p].nx * h->hp[p].ny);
    h->stage_len = (size_t)maxcells * nv;
    TRY(([&]() -> int { HIP_TRY(h, dalloc(&h->stage, h->stage_len)); return 0; })());
    const hipMemcpyKind kind = device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int p = 0; p < nprob; ++p) {
        const long long n = (long long)h->hp[p].nx * h->hp[p].ny;
        const int nblk = (int)((n + 255) / 256);
        const double* srcs[3] = {W0[p], Wx0[p], dim == 2 ? Wy0[p] : nullptr};
        double* dsts[3] = {h->W, h->Wx, h->Wy};
        for (int a = 0; a < (dim == 2 ? 3 : 2); ++a) {
            TRY(([&]() -> int {
                HIP_TRY(h, hipMemcpyAsync(h->stage, srcs[a], sizeof(double) * n * nv, kind, h->stream));
                aos_to_soa<<<nblk, 256, 0, h->stream>>>(h->stage, dsts[a] + h->hp[p].coff, n, nv, N);
                HIP_TRY(h, hipGetLastError());
                HIP_TRY(h, hipStreamSynchronize(h->stream));
                return 0;
            })());
        }
    }
    // first dt from the initial state
    if (dim == 1)
        gks::signal1d_kernel<<<h->nTilesC, gks::kBlock1D, 0, h->stream>>>(h->dP, h->dS, h->dTilesC, h->W, h->Ntot);
    else
        gks::signal2d_kernel<<<dim3((probs[0].nx + 63) / 64, (probs[0].ny + 3) / 4), dim3(64, 4), 0, h->stream>>>(
            h->dP, h->dS, h->W);
    gks::finish_kernel<<<(nprob + 63) / 64, 64, 0, h->stream>>>(h->dP, h->dS, nprob, 0, h->ctr, dim == 1 ? 3 : 2);
    std::vector<ProbState> s(nprob);
    TRY(([&]() -> int {
        HIP_TRY(h, hipGetLastError());
        HIP_TRY(h, hipMemcpyAsync(s.data(), h->dS, sizeof(ProbState) * nprob, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        return 0;
    })());
    for (int p = 0; p < nprob; ++p)
        if (s[p].err) {
            h->err = "problem " + std::to_string(p) + ": non-physical initial state";
            return bail(GKS_EINVAL);
        }
#undef TRY
    *out = h;
    return GKS_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free 1-D run (gks_run1d_noalloc): every buffer the batched 1-D
// kernels use lives in `scratch`, a static device array of the library
// (each GPU holds its own copy until the process ends).  Host code never
// passes the array's name to a kernel: the address comes from
// hipGetSymbolAddress, taken once per device.
// ---------------------------------------------------------------------------
constexpr long long kNoAllocMaxCells = 32768;
constexpr int kNoAllocBlk = 256;                                     // tile: 255 cells per work item
constexpr long long kNoAllocItems = kNoAllocMaxCells / (kNoAllocBlk - 1) + 1;
constexpr long long kNoAllocTilesC = kNoAllocMaxCells / gks::kBlock1D + 1;
// layout (in doubles, every part 256-byte aligned)
constexpr long long na_round(long long d) { return (d + 31) & ~31ll; }
constexpr long long kNaPar = 0;
constexpr long long kNaState = kNaPar + na_round((sizeof(ProbParam) + 7) / 8);
constexpr long long kNaCtr = kNaState + na_round((sizeof(ProbState) + 7) / 8); // 3 counters + item count
constexpr long long kNaAll = kNaCtr + 32;
constexpr long long kNaAct = kNaAll + na_round(kNoAllocItems);                 // Tile = 8 bytes
constexpr long long kNaFirst = kNaAct + na_round(kNoAllocItems);               // first[1], count[1]
constexpr long long kNaTilesC = kNaFirst + 32;
constexpr long long kNaW = kNaTilesC + na_round(kNoAllocTilesC);
constexpr long long kNaWx = kNaW + na_round(9 * kNoAllocMaxCells);
constexpr long long kNaPW = kNaWx + na_round(9 * kNoAllocMaxCells);
constexpr long long kNaPf = kNaPW + na_round(3 * kNoAllocMaxCells);
constexpr long long kScratchDoubles = kNaPf + na_round(3 * (kNoAllocMaxCells + 1));

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mutex;

// the device address of this device's scratch array (taken once per device)
hipError_t scratch_address(int dev, double** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Set-up of a run in the scratch area: the problem's parameters and state
// (time t0, active), cleared counters, the full work-item list of BLK - 1
// cells per item and the 128-cell tiles of the signal-speed kernel.
__global__ void noalloc_setup(ProbParam P, double t0, ProbParam* dP, ProbState* dS, unsigned* ctr, int* nact,
                              Tile* all, int* first, int* count, Tile* tilesC, int nitems, int ntiles)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *dP = P;
        ProbState S{};
        S.t = t0;
        S.active = 1;
        *dS = S;
        ctr[0] = ctr[1] = ctr[2] = 0u;
        *nact = 0;
        first[0] = 0;
        count[0] = nitems;
    }
    if (i < nitems) all[i] = Tile{0, i * (kNoAllocBlk - 1)};
    if (i < ntiles) tilesC[i] = Tile{0, i * gks::kBlock1D};
}

// state slot holding W^n -> caller's [nx][3] arrays
__global__ void noalloc_out(const ProbState* __restrict__ dS, const double* __restrict__ W,
                            const double* __restrict__ Wx, double* __restrict__ Wo, double* __restrict__ Wxo, long long n)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const size_t base = (size_t)dS->cur * 3 * n;
    for (int k = 0; k < 3; ++k) {
        Wo[c * 3 + k] = W[base + k * n + c];
        Wxo[c * 3 + k] = Wx[base + k * n + c];
    }
}

template <typename T>
void noalloc_steps(const ProbParam* dP, ProbState* dS, Tile* act, int* nact, unsigned* ctr, double* W, double* Wx,
                   double* PW, double* Pf, long long N, long long F, Tile* all, int* first, int* count, int G,
                   int nsteps, hipStream_t st)
{
    for (int s = 0; s < nsteps; ++s) {
        gks::stage1d_kernel<T, 1, kNoAllocBlk><<<G, kNoAllocBlk, 0, st>>>(dP, dS, act, nact, ctr, W, Wx, PW, Pf, N, F);
        gks::stage1d_kernel<T, 2, kNoAllocBlk><<<G, kNoAllocBlk, 0, st>>>(dP, dS, act, nact, ctr, W, Wx, PW, Pf, N, F);
        gks::commit1d_kernel<<<1, gks::kPhaseBlk, 0, st>>>(dP, dS, act, nact, ctr, 1, all, first, count);
    }
}

} // namespace

extern "C" {

int gks_init(const gks_problem* probs, int32_t nprob, int32_t precision, const double* const* W0,
             const double* const* Wx0, const double* const* Wy0, void* stream, gks_handle** out)
{
    return init_common(probs, nprob, precision, W0, Wx0, Wy0, stream, out, false);
}

int gks_init_device(const gks_problem* probs, int32_t nprob, int32_t precision, const double* const* W0,
                    const double* const* Wx0, const double* const* Wy0, void* stream, gks_handle** out)
{
    return init_common(probs, nprob, precision, W0, Wx0, Wy0, stream, out, true);
}

int gks_step(gks_handle* h, int32_t max_steps, int32_t* n_active)
{
    if (!h) return fail(nullptr, GKS_EINVAL, "NULL handle");
    if (h->dead) return dead_handle(h);
    if (max_steps < 0) return fail(h, GKS_EINVAL, "max_steps < 0");
    std::vector<ProbState> before(h->nprob), after(h->nprob);
    HIP_TRY(h, hipMemcpyAsync(before.data(), h->dS, sizeof(ProbState) * h->nprob, hipMemcpyDeviceToHost, h->stream));
    if (!h->tuned && max_steps > 0) {
        const int st = autotune(h);
        if (st) return st;
    }
    if (h->dim == 1 && h->tuned) {
        // lane-pair steps while the work items of the tuned tile size still
        // running (known from the last call) are at most half the CUs, so
        // the lane-pair items (twice as many) still fill each CU once
        int want = h->split_mode == 2;
        if (h->split_mode == 1) {
            const int bn = h->blk == 64 ? 0 : (h->blk == 128 ? 1 : 2);
            long long items = 0;
            for (int p = 0; p < h->nprob; ++p)
                if (h->last_active[p]) items += h->hcount[bn][p];
            want = 2 * items <= h->ncu;
        }
        // two-kernel steps while the 255-cell items fill the CUs several
        // times; the lane-pair steps take precedence
        int wantp = 0;
        if (!want && h->phases_mode != 0) {
            long long items = 0;
            for (int p = 0; p < h->nprob; ++p)
                if (h->last_active[p]) items += h->hcount[2][p];
            wantp = h->phases_mode == 2 || items >= kPhaseItemsPerCU * h->ncu;
        }
        if (wantp && !h->R1) {
            // the face buffer, allocated on first use; without it the steps
            // stay fused
            if (dalloc(&h->R1, 21 * (size_t)h->F) != hipSuccess) {
                (void)hipGetLastError();
                h->R1 = nullptr;
                h->phases_mode = 0;
                wantp = 0;
            }
        }
        if (want != h->split || wantp != h->phases) {
            h->split = want;
            h->phases = wantp;
            drop_graph(h);
        }
    }
    const bool graph = h->use_graph && !h->timing && max_steps > 0;
    if (graph && !h->gexec[0]) {
        const int st = build_graph(h);
        if (st) return st;
    }
    int s = 0;
    if (graph)
        for (int g = 2; g >= 1; --g)
            for (; s + kGraphSteps[g - 1] <= max_steps; s += kGraphSteps[g - 1])
                HIP_TRY(h, hipGraphLaunch(h->gexec[g], h->stream));
    for (; s < max_steps; ++s) {
        if (graph) HIP_TRY(h, hipGraphLaunch(h->gexec[0], h->stream));
        else launch_step(h, h->stream);
    }
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipMemcpyAsync(after.data(), h->dS, sizeof(ProbState) * h->nprob, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    harvest(h);
    int active = 0, bad = -1;
    long long upd = 0;
    for (int p = 0; p < h->nprob; ++p) {
        active += after[p].active;
        h->last_active[p] = after[p].active ? 1 : 0;
        if (after[p].err && !before[p].err && bad < 0) bad = p;
        upd += (after[p].nsteps - before[p].nsteps) * (long long)h->hp[p].nx * h->hp[p].ny;
    }
    h->last_updates = upd;
    if (n_active) *n_active = active;
    if (bad >= 0) {
        char buf[160];
        snprintf(buf, sizeof buf, "problem %d: non-physical state at t = %.17g (step %lld)", bad, after[bad].t,
                 after[bad].nsteps);
        return fail(h, GKS_ENONPHYS, buf);
    }
    return GKS_OK;
}

static int state_common(const gks_handle* hc, int32_t p, double* W, double* Wx, double* Wy, bool device)
{
    gks_handle* h = const_cast<gks_handle*>(hc);
    if (!h) return fail(nullptr, GKS_EINVAL, "NULL handle");
    if (h->dead) return dead_handle(h);
    if (p < 0 || p >= h->nprob) return fail(h, GKS_EINVAL, "problem index out of range");
    ProbState& s = h->last_state;
    HIP_TRY(h, hipMemcpyAsync(&s, h->dS + p, sizeof s, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const ProbParam& P = h->hp[p];
    const long long n = (long long)P.nx * P.ny;
    const int nv = h->dim + 2;
    const long long N = h->Ntot;
    const int nblk = (int)((n + 255) / 256);
    double* srcs[3] = {h->W, h->Wx, h->Wy};
    double* dsts[3] = {W, Wx, Wy};
    const hipMemcpyKind kind = device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int a = 0; a < (h->dim == 2 ? 3 : 2); ++a) {
        if (!dsts[a]) continue;
        soa_to_aos<<<nblk, 256, 0, h->stream>>>(srcs[a] + (size_t)s.cur * nv * N + P.coff, h->stage, n, nv, N);
        HIP_TRY(h, hipGetLastError());
        HIP_TRY(h, hipMemcpyAsync(dsts[a], h->stage, sizeof(double) * n * nv, kind, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    return GKS_OK;
}

int gks_state(const gks_handle* hc, int32_t p, double* W, double* Wx, double* Wy, double* t, int64_t* nsteps)
{
    int st = state_common(hc, p, W, Wx, Wy, false);
    if (st) return st;
    const ProbState& s = hc->last_state; // read by state_common on the handle's stream
    if (t) *t = s.t;
    if (nsteps) *nsteps = s.nsteps;
    return GKS_OK;
}

int gks_state_device(const gks_handle* h, int32_t p, double* W, double* Wx, double* Wy)
{
    return state_common(h, p, W, Wx, Wy, true);
}

int gks_problem_status(const gks_handle* hc, int32_t p, int32_t* status)
{
    gks_handle* h = const_cast<gks_handle*>(hc);
    if (!h || !status) return fail(h, GKS_EINVAL, "NULL argument");
    if (h->dead) return dead_handle(h);
    if (p < 0 || p >= h->nprob) return fail(h, GKS_EINVAL, "problem index out of range");
    ProbState s;
    HIP_TRY(h, hipMemcpyAsync(&s, h->dS + p, sizeof s, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    *status = s.err ? GKS_ENONPHYS : (s.active ? 0 : 1);
    return GKS_OK;
}

int gks_free(gks_handle* h)
{
    release(h);
    return GKS_OK;
}

const char* gks_last_error(const gks_handle* h)
{
    return h ? h->err.c_str() : g_init_error.c_str();
}

int gks_kernel_timing(gks_handle* h, int32_t enable)
{
    if (!h) return fail(nullptr, GKS_EINVAL, "NULL handle");
    h->timing = enable != 0;
    for (int k = 0; k < 3; ++k) { h->tot_ms[k] = 0.0; h->launches[k] = 0; }
    return GKS_OK;
}

int gks_kernel_time(gks_handle* h, int32_t kernel_id, double* total_ms, int64_t* launches)
{
    if (!h || kernel_id < 0 || kernel_id > 2) return fail(h, GKS_EINVAL, "bad kernel id");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    harvest(h);
    if (total_ms) *total_ms = h->tot_ms[kernel_id];
    if (launches) *launches = h->launches[kernel_id];
    return GKS_OK;
}

const char* gks_launch_config(const gks_handle* hc)
{
    if (!hc) return "";
    gks_handle* h = const_cast<gks_handle*>(hc);
    if (h->dim == 2) {
        h->cfg_text = "2-D: fixed tiles (face rows 64x4, Gauss points 64x4, cells 64x4)";
    } else if (!h->tuned) {
        h->cfg_text = "1-D: not tuned yet (tunes on the first gks_step)";
    } else {
        const int n = h->nItems[h->blk == 64 ? 0 : (h->blk == 128 ? 1 : 2)];
        char buf[320];
        snprintf(buf, sizeof buf,
                 "; blk %d gmul %d: %d workgroups for %d work items; lane-pair steps %s (%s); two-kernel steps %s (%s)",
                 h->blk, h->gmul, h->gmul == 0 ? n : std::min(n, h->gmul * h->ncu), n, h->split ? "on" : "off",
                 h->split_mode == 0 ? "never" : (h->split_mode == 2 ? "always" : "while items <= CUs / 2"),
                 h->phases ? "on" : "off",
                 h->phases_mode == 0 ? "never" : (h->phases_mode == 2 ? "always" : "while 255-cell items >= 2 per CU"));
        h->cfg_text = h->tune_note + buf;
    }
    return h->cfg_text.c_str();
}

int gks_cell_updates(const gks_handle* h, int64_t* count)
{
    if (!h || !count) return GKS_EINVAL;
    *count = h->last_updates;
    return GKS_OK;
}

int gks_run1d_noalloc(const gks_problem* prob, int32_t precision, double* W, double* Wx, int32_t nsteps, double t0,
                      void* stream, double* t_out, int64_t* steps_out, int32_t* status_out)
{
    if (!prob || !W || !Wx || nsteps < 0) return fail(nullptr, GKS_EINVAL, "gks_run1d_noalloc: NULL argument or nsteps < 0");
    int st = validate(prob, 1, precision);
    if (st) return st;
    if (prob->dim != 1) return fail(nullptr, GKS_EINVAL, "gks_run1d_noalloc: 1-D problems only");
    if (prob->nx > kNoAllocMaxCells) {
        char buf[160];
        snprintf(buf, sizeof buf, "gks_run1d_noalloc: %d cells exceed the scratch limit of %lld cells", prob->nx,
                 kNoAllocMaxCells);
        return fail(nullptr, GKS_EINVAL, buf);
    }
    if (!std::isfinite(t0)) return fail(nullptr, GKS_EINVAL, "gks_run1d_noalloc: t0 must be finite");
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) return fail(nullptr, GKS_EDEVICE, "device index out of range");
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    double* base = nullptr;
    if (e == hipSuccess) e = scratch_address(dev, &base);
    if (e != hipSuccess) return fail(nullptr, GKS_EDEVICE, std::string("gks_run1d_noalloc: ") + hipGetErrorString(e));
    hipStream_t s = (hipStream_t)stream;
    const long long N = prob->nx, F = N + 1;
    ProbParam* dP = reinterpret_cast<ProbParam*>(base + kNaPar);
    ProbState* dS = reinterpret_cast<ProbState*>(base + kNaState);
    unsigned* ctr = reinterpret_cast<unsigned*>(base + kNaCtr);
    int* nact = reinterpret_cast<int*>(ctr + 3);
    Tile* all = reinterpret_cast<Tile*>(base + kNaAll);
    Tile* act = reinterpret_cast<Tile*>(base + kNaAct);
    int* first = reinterpret_cast<int*>(base + kNaFirst);
    int* count = first + 1;
    Tile* tilesC = reinterpret_cast<Tile*>(base + kNaTilesC);
    double *dW = base + kNaW, *dWx = base + kNaWx, *dPW = base + kNaPW, *dPf = base + kNaPf;
    const int nitems = (int)((N + kNoAllocBlk - 2) / (kNoAllocBlk - 1));
    const int ntiles = (int)((N + gks::kBlock1D - 1) / gks::kBlock1D);
    const int nb = (int)((N + 255) / 256);
    // parameters, state, counters and work lists; the caller's arrays into slot 0
    noalloc_setup<<<std::max(1, (std::max(nitems, ntiles) + 255) / 256), 256, 0, s>>>(
        make_param(*prob, 1, 0, 0), t0, dP, dS, ctr, nact, all, first, count, tilesC, nitems, ntiles);
    aos_to_soa<<<nb, 256, 0, s>>>(W, dW, N, 3, N);
    aos_to_soa<<<nb, 256, 0, s>>>(Wx, dWx, N, 3, N);
    // first dt from the state, the active work list, then the steps
    gks::signal1d_kernel<<<ntiles, gks::kBlock1D, 0, s>>>(dP, dS, tilesC, dW, N);
    gks::finish_kernel<<<1, 64, 0, s>>>(dP, dS, 1, 0, ctr, 3);
    gks::compact_items_kernel<<<1, gks::kCompactThreads, 0, s>>>(dS, 1, all, first, count, act, nact);
    const int G = std::min(nitems, std::max(ncu, 1));
    if (precision == GKS_PREC_FP64)
        noalloc_steps<double>(dP, dS, act, nact, ctr, dW, dWx, dPW, dPf, N, F, all, first, count, G, nsteps, s);
    else
        noalloc_steps<float>(dP, dS, act, nact, ctr, dW, dWx, dPW, dPf, N, F, all, first, count, G, nsteps, s);
    noalloc_out<<<nb, 256, 0, s>>>(dS, dW, dWx, W, Wx, N);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, GKS_EDEVICE, std::string("gks_run1d_noalloc: ") + hipGetErrorString(e));
    if (t_out || steps_out || status_out) {
        ProbState S{};
        e = hipMemcpyAsync(&S, dS, sizeof S, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(nullptr, GKS_EDEVICE, std::string("gks_run1d_noalloc: ") + hipGetErrorString(e));
        if (t_out) *t_out = S.t;
        if (steps_out) *steps_out = S.nsteps;
        if (status_out) *status_out = S.err ? GKS_ENONPHYS : (S.active ? 0 : 1);
    }
    return GKS_OK;
}

} // extern "C"
