/*
 * gks.h -- C ABI of the MI355X (gfx950) library for the compact 6th/8th-order
 * gas-kinetic scheme of Zhao, Ji, Shyy and Xu (arXiv:1901.00261).
 *
 * The library advances cell averages W and cell-averaged gradients W_x (and
 * W_y) of the Euler / Navier-Stokes equations on uniform meshes with the
 * two-stage fourth-order multi-stage multi-derivative (MSMD) time stepping
 * (Sec. 2.2), compact linear reconstruction for the equilibrium state
 * (Sec. 3.1), compact WENO-Z for the non-equilibrium state (Sec. 3.3) and the
 * simplified third-order BGK interface distribution (Sec. 2.1).
 *
 * Conventions
 *   - Every call returns an int status: GKS_OK (0) or a negative GKS_E*.
 *     Errors never abort the process; gks_last_error() explains the last one.
 *   - Host arrays are row-major [ny][nx][nv], nv = dim + 2, conservative
 *     variables (rho, rho U, [rho V], rho E); gradients are cell-averaged
 *     gradients (not multiplied by the cell width).  The library copies them;
 *     the caller keeps ownership.
 *   - A handle is not re-entrant: calls on one handle must not overlap.
 *     Separate handles are independent.
 *   - All device work runs on the stream given to gks_init (a hipStream_t;
 *     NULL means the library creates its own default-priority stream).
 *   - The library links the HIP runtime by its soname (libamdhip64.so.7).  In
 *     a process that also uses another copy of the runtime (PyTorch bundles
 *     one), load that copy first so that this library binds to it: streams
 *     and device buffers are then shared by one runtime.
 */
#ifndef GKS_H
#define GKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GKS_OK = 0,
    GKS_EINVAL = -1,   /* invalid argument */
    GKS_ENOMEM = -2,   /* device allocation failed */
    GKS_EDEVICE = -3,  /* HIP runtime error */
    GKS_ENONPHYS = -4, /* a non-physical state (rho <= 0 or p <= 0) was met */
    GKS_ESTATE = -5    /* handle unusable: a HIP runtime call failed on it earlier (that call returned
                          GKS_EDEVICE or GKS_ENOMEM); only gks_free and gks_last_error remain useful */
};
/* Boundary conditions, per side (Sec. 4 uses periodic, non-reflecting,
   reflecting-wall and prescribed-state boundaries).
   Periodic: wrap (both sides of a direction).
   Extrapolated (the paper's non-reflecting ends): ghost cells copy the
     boundary cell with zero normal slope.
   Reflecting wall: ghost cells are the mirror image of the interior (normal
     momentum negated; normal slopes of the other variables negated).
   Inflow: ghost cells hold the side's state A (bc_state) with zero slopes.
   Split (2-D only; the double Mach reflection of Sec. 4.5): ghost cells at
     position s along the side (cell-centre coordinate) hold state A where
     s < bc_split[0] + bc_split[1] * t, and beyond that point are a
     reflecting wall (bc_beyond = GKS_BC_REFLECT) or hold state B
     (bc_beyond = GKS_BC_INFLOW); t is the time of the stage.
   Characteristic (1-D only): the boundary cell is projected on the Euler
     eigenvectors at its state; fields leaving the domain are extended
     linearly with their slopes, incoming fields keep the boundary value
     with zero slope.
   Where two sides meet, the corner ghosts follow the y sides. */
enum { GKS_BC_PERIODIC = 0, GKS_BC_EXTRAP = 1, GKS_BC_REFLECT = 2, GKS_BC_INFLOW = 3, GKS_BC_SPLIT = 4,
       GKS_BC_CHAR = 5 };
enum { GKS_RECON_LINEAR = 0, GKS_RECON_WENOZ = 1 };
enum { GKS_PREC_FP64 = 0, GKS_PREC_FP32_MIXED = 1 };

/* One problem (Sec. 2 and Sec. 4 of the paper).
   dim: 1 or 2.  nx, ny: interior cells (ny = 1 when dim == 1), at least 4.
   gamma > 1.  mu >= 0 dynamic viscosity (0: Euler); collision times follow
   Sec. 4: the viscous terms take mu/p (0 for Euler) plus the pressure-jump
   term |p_l - p_r| / (p_l + p_r) dt, the exponentials eps dt (Euler,
   eps = 0.01) or mu/p plus the same jump term.  cfl > 0 sets
   dt = cfl * min over cells of dx/(|U|+c) [and dy/(|V|+c)] unless
   dt_fixed > 0.  The last step is shortened so the problem ends exactly at
   t_end.  order: 6 or 8.  recon: GKS_RECON_*.  bc: x-low, x-high, y-low,
   y-high, GKS_BC_* (periodic must be paired).  bc_state[side][0/1]: the
   inflow states A and B of a side, conservative (rho, rho U, rho V, rho E)
   (rho V ignored in 1-D; must be physical where used); bc_split[side]: the
   switch position at t = 0 and its speed; bc_beyond[side]: GKS_BC_REFLECT
   or GKS_BC_INFLOW (split sides only).  Fields of sides that do not use
   them are ignored (zero-initialise them). */
typedef struct {
    int32_t dim;
    int32_t nx, ny;
    double xlo, xhi, ylo, yhi;
    double gamma;
    double mu;
    double cfl;
    double dt_fixed;
    double t_end;
    int32_t order;
    int32_t recon;
    int32_t bc[4];
    double bc_state[4][2][4];
    double bc_split[4][2];
    int32_t bc_beyond[4];
} gks_problem;

typedef struct gks_handle gks_handle;

/* Create a handle holding nprob problems, all of the same dim (2-D handles
   hold one problem).  W0[p], Wx0[p], Wy0[p] are host arrays (Wy0 may be NULL
   when dim == 1).  precision: GKS_PREC_*.  stream: hipStream_t or NULL.
   On success *out owns device memory until gks_free.
   Errors: GKS_EINVAL (bad sizes/parameters, non-physical initial data),
   GKS_ENOMEM, GKS_EDEVICE. */
int gks_init(const gks_problem* probs, int32_t nprob, int32_t precision, const double* const* W0,
             const double* const* Wx0, const double* const* Wy0, void* stream, gks_handle** out);

/* Same as gks_init with DEVICE pointers (for example torch tensors on the
   GPU); the library copies them device-to-device on its stream. */
int gks_init_device(const gks_problem* probs, int32_t nprob, int32_t precision, const double* const* W0,
                    const double* const* Wx0, const double* const* Wy0, void* stream, gks_handle** out);

/* Advance every unfinished problem by up to max_steps MSMD steps, each with
   its own dt (Sec. 2.2).  *n_active (may be NULL) receives the number of
   problems still short of t_end.  Returns GKS_ENONPHYS if any problem met a
   non-physical state; that problem stops and keeps the state it had at the
   start of the failing step.  All max_steps steps are launched (finished
   problems skip their work but the launches still cost time), so a caller
   running to t_end steps in chunks; multiples of 8 keep the eight-step graph
   replays. */
int gks_step(gks_handle* h, int32_t max_steps, int32_t* n_active);

/* Copy problem p to host buffers (layout as in gks_init; Wy ignored when
   dim == 1) and report its time and step count (either may be NULL).
   Synchronises the stream. */
int gks_state(const gks_handle* h, int32_t p, double* W, double* Wx, double* Wy, double* t, int64_t* nsteps);

/* Same as gks_state into DEVICE buffers (no host synchronisation beyond the
   stream order). */
int gks_state_device(const gks_handle* h, int32_t p, double* W, double* Wx, double* Wy);

/* Status of problem p: 0 running, 1 finished (t == t_end), GKS_ENONPHYS. */
int gks_problem_status(const gks_handle* h, int32_t p, int32_t* status);

int gks_free(gks_handle* h);

/* Message of the last failure on h (or of the last failed gks_init when h is
   NULL).  Static lifetime until the next call on the same handle. */
const char* gks_last_error(const gks_handle* h);

/* Kernel timing with HIP events on the handle's stream.  enable != 0 records
   an event pair around every launch of the kernels of the given id from now
   on; gks_kernel_time returns the summed time (ms) and the launch count since
   enabling.  Ids: 0 interface (flux) kernels (1-D: the pair of fused stage
   kernels, interface and cell update, counts as one launch), 1 face-row
   reconstruction kernels (2-D), 2 cell update kernels (2-D).  Steps are not
   replayed from a graph while timing is on. */
int gks_kernel_timing(gks_handle* h, int32_t enable);
int gks_kernel_time(gks_handle* h, int32_t kernel_id, double* total_ms, int64_t* launches);

/* Number of cells * MSMD steps the last gks_step performed (all problems). */
int gks_cell_updates(const gks_handle* h, int64_t* count);

/* Launch configuration of the handle (text, valid until the next call on
   h).  A batched 1-D handle runs one kernel per MSMD stage over work items
   of BLK-1 cells (BLK = 64, 128 or 256 threads), with GMUL persistent
   workgroups per compute unit or, for GMUL = 0, one workgroup per item.
   The first gks_step of a 1-D handle autotunes (BLK, GMUL) by timing a few
   steps from the initial state, which is restored afterwards (larger tiles
   and fewer workgroups are tried first and kept unless another candidate
   is more than 3 % faster).  Each gks_step call chooses the form of its
   steps from the work items still active after the previous call: at most
   half as many 127-cell items as compute units, a lane-pair kernel (two
   lanes per face); at least two 255-cell items per compute unit, two
   kernels per stage (face reconstruction; interface point and cells);
   otherwise the tuned kernel.  Every configuration and form performs the
   same arithmetic, so results do not depend on the choice.  Environment:
   GKS_TUNE="BLK:GMUL" forces a configuration, GKS_TUNE_CACHE=<file> caches
   tuning results by problem-set signature, GKS_GRAPH=0 disables the
   hipGraph replay of steps (enabled by default), GKS_SPLIT and GKS_PHASES
   (0 never, 1 automatic, the default, 2 always) control the lane-pair and
   two-kernel forms. */
const char* gks_launch_config(const gks_handle* h);

/* For callers that cannot allocate device memory: code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc.  Advances
   ONE 1-D problem (prob->dim == 1, at most GKS_NOALLOC_MAX_CELLS cells) by
   nsteps MSMD steps, starting at time t0, in place in the caller's DEVICE
   arrays W and Wx ([nx][3] row-major, as gks_init_device takes them), with
   the same kernels and arithmetic as gks_step.  All working storage (state
   slots, MSMD partials, parameters, work lists) is a static device array of
   the library, one per GPU, held until the process ends: the call performs
   no allocation, memset or host-to-device copy; it only enqueues kernels on
   `stream` (a hipStream_t; NULL: the default stream) and returns.  Only when
   t_out, steps_out or status_out is non-NULL does it also copy the run's
   final time, its step count and its status (0 running, 1 reached t_end,
   GKS_ENONPHYS) to the host and synchronise the stream.  A problem that
   meets a non-physical state stops there; W and Wx then hold the state at
   the start of the failing step.  Every call on a GPU shares that GPU's
   static array, and each call re-initialises what it uses: calls that
   overlap on one GPU (different streams or host threads) race and must not
   be issued.  Errors: GKS_EINVAL (invalid problem, 2-D, more than
   GKS_NOALLOC_MAX_CELLS cells, nsteps < 0), GKS_EDEVICE. */
#define GKS_NOALLOC_MAX_CELLS 32768
int gks_run1d_noalloc(const gks_problem* prob, int32_t precision, double* W, double* Wx, int32_t nsteps, double t0,
                      void* stream, double* t_out, int64_t* steps_out, int32_t* status_out);

#ifdef __cplusplus
}
#endif

#endif /* GKS_H */
