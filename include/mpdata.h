/*
 * mpdata.h -- C ABI of libmpdata.so: the MPDATA advection step on a 3-D
 * structured grid, as hand-written HIP kernels for MI355X (gfx950).
 *
 * The operation (paper: ESCAPE D2.5, Section 5, the MPDATA dwarf):
 *   one time step of  d(G psi)/dt + div(V psi) = 0  made of
 *   - a donor-cell (upwind) pass: the upwind face flux of Listings 4-5, its
 *     vertical counterpart of Listings 6-7 (a closed axis is the boundary
 *     factor 0 there), the flux divergence over the cell's metric volume and
 *     the solution update of Listing 8;
 *   - (iters - 1) antidiffusive corrective passes (the MPDATA iterations the
 *     paper refers to its companion deliverable), each optionally limited by
 *     the non-oscillatory (flux-corrected transport) limiter.
 *
 * Arrays.  psi, g, cx, cy, cz are dense C-order [nz][ny][nx] arrays (i
 * fastest) of the problem's dtype, in DEVICE memory, contiguous and naturally
 * aligned.  Staggered face arrays share the cell index space (the C-grid
 * convention of Section 3.1.4.1): cx[k][j][i] is the Courant number on face
 * (i+1/2, j, k), cy on (i, j+1/2, k), cz on (i, j, k+1/2).  On a periodic axis
 * the last slot is the wrap face n-1/2 == -1/2.  On a closed axis the faces
 * -1/2 and n-1/2 carry no flux and the slot n-1 is never read.  g is the
 * metric (cell volume factor, the paper's dual volume times density).
 *
 * Input ranges (preconditions, not checked unless MPDATA_DEBUG is set):
 *   psi in [0, 1e100] in FP64, [0, 1e30] in FP32 (the sign-preserving form of
 *       the scheme needs psi >= 0; the upper bound keeps the fused pass's
 *       products of three guarded pair sums finite);
 *   g in [1e-6, 1e6];
 *   |Courant numbers| small enough for the donor-cell bound (the outflow
 *       Courant sum of a cell over its g at most 1) for positivity.
 * Within these ranges (and eps as below) every result is finite.
 *
 * MPDATA_DEBUG.  With the environment variable MPDATA_DEBUG set (to anything
 * but "0"), mpdata_step, mpdata_run, mpdata_adjoint and mpdata_run_batched
 * scan psi and g on the device before enqueueing the step and return
 * MPDATA_EINVAL if a value lies outside the ranges above or is NaN.  The scan
 * synchronises the stream; it is skipped while the stream is being captured.
 *
 * Ownership.  The caller owns every buffer, including the workspace, whose
 * size mpdata_workspace_bytes() returns.  These calls never allocate device
 * memory.  psi_in must not alias psi_out (MPDATA_EINVAL).
 *
 * Errors.  Every call validates its arguments synchronously, before anything
 * is enqueued, and returns MPDATA_OK or a negative code; the reason is then
 * in mpdata_last_error() (thread-local, valid until the next call on the same
 * thread).  A failed launch returns MPDATA_EDEVICE.  Faults inside a kernel
 * surface at the caller's next synchronisation.
 *
 * Asynchrony.  Work is enqueued on `stream` (a hipStream_t; NULL = the null
 * stream) and the calls return after enqueueing, except mpdata_mass, which
 * synchronises the stream.  Forward calls are bitwise reproducible (no
 * atomics).
 */
#ifndef MPDATA_H
#define MPDATA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MPDATA_OK = 0,
    MPDATA_EINVAL = -1,       /* invalid argument (a workspace below the size */
                              /* the query returns included), see             */
                              /* mpdata_last_error()                          */
    MPDATA_ENOMEM = -2,       /* reserved; not returned by these calls        */
    MPDATA_EDEVICE = -3,      /* HIP launch or runtime error                  */
    MPDATA_EUNSUPPORTED = -4  /* valid but not implemented combination        */
};

enum { MPDATA_F64 = 0, MPDATA_F32 = 1 };
enum { MPDATA_PERIODIC = 0, MPDATA_CLOSED = 1 };
enum { MPDATA_OP_STEP = 0, MPDATA_OP_RUN = 1, MPDATA_OP_ADJOINT = 2, MPDATA_OP_MASS = 3 };

typedef struct {
    int32_t nx, ny, nz;   /* cells per axis, each >= 1; nz == 1 is a 2-D problem  */
    int32_t bc[3];        /* per axis x, y, z: MPDATA_PERIODIC or MPDATA_CLOSED    */
    int32_t iters;        /* passes per step, 1..8: 1 = donor cell only,          */
                          /* 2 = donor cell + 1 corrective pass, ...              */
    int32_t limiter;      /* 0 = off, 1 = non-oscillatory limiter on              */
    int32_t dtype;        /* MPDATA_F64 or MPDATA_F32 (storage and arithmetic)    */
    int32_t reserved;     /* must be 0                                            */
    double eps;           /* denominator guard of the antidiffusive and limiter   */
                          /* ratios: 0 selects 1e-15, else in [1e-30, 1e-3]      */
                          /* (the floor keeps every guarded denominator normal   */
                          /* in both precisions)                                 */
} mpdata_problem;

/* Workspace bytes for `op` (MPDATA_OP_*).  nsteps and checkpoint_every matter
 * for MPDATA_OP_ADJOINT only.  Returns 0 and sets the error text if p is
 * invalid. */
size_t mpdata_workspace_bytes(const mpdata_problem* p, int32_t op, int32_t nsteps,
                              int32_t checkpoint_every);

/* One step: psi_out = step(psi_in).  cz may be NULL (all vertical Courant
 * numbers 0).  ws: device workspace of ws_bytes >= the MPDATA_OP_STEP size. */
int mpdata_step(const mpdata_problem* p, const void* psi_in, void* psi_out,
                const void* cx, const void* cy, const void* cz, const void* g,
                void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the step
 * of mpdata_step, with its workspace taken from a fixed device array of
 * MPDATA_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs
 * on until the process ends, instead of a caller's buffer.  The call
 * allocates no device memory (its first call on a device looks the array's
 * address up).  A problem whose MPDATA_OP_STEP workspace exceeds the array
 * (FP64: up to ~2.1 M cells, e.g. 256 x 128 x 64; FP32: twice that) is
 * refused with MPDATA_EINVAL.  All calls on one GPU share that GPU's array
 * and leave their intermediates in it: calls that overlap on one GPU (on
 * concurrent streams or from several threads) race and their results are
 * undefined, so the caller serialises them.  Arguments, errors and
 * asynchrony as mpdata_step. */
#define MPDATA_NOALLOC_SCRATCH_BYTES (168u << 20)
int mpdata_step_noalloc(const mpdata_problem* p, const void* psi_in, void* psi_out, const void* cx,
                        const void* cy, const void* cz, const void* g, void* stream);

/* nsteps >= 0 steps in place: psi holds psi^0 on entry and psi^nsteps on
 * return (after the stream has run).  Winds and metric are the same for all
 * steps.  ws: at least the MPDATA_OP_RUN size. */
int mpdata_run(const mpdata_problem* p, int32_t nsteps, void* psi,
               const void* cx, const void* cy, const void* cz, const void* g,
               void* ws, size_t ws_bytes, void* stream);

/* Adjoint (reverse mode) of mpdata_run, FP64 only.  For a cost J(psi_T) of
 * the state after nsteps steps, takes the seed dJ_dpsiT = dJ/dpsi_T and
 * returns dJ/dpsi0 and dJ/d(cx, cy, cz) (dJ_dcz may be NULL to skip it; the
 * closed-wall slots of the gradients are 0).  The forward trajectory is
 * recomputed from psi0: states are kept every checkpoint_every steps (0 =
 * only psi0) and each segment is recomputed before its reverse sweep, its
 * steps storing the intermediates the reverse sweep reads (the forward
 * sweep runs the same kernels, so the result does not depend on
 * checkpoint_every; psiT_out agrees with mpdata_run to rounding).  At
 * the kinks of max/min the derivative follows the branch the forward step
 * took ([c]+ differentiates to [c > 0], 1/2 at c = 0, |c| to sign(c) with sign(0) = 0,
 * min(1, min(a, b)) to its first minimal entry, the limiter bounds to their
 * first extremal entry).  psiT_out (nullable) receives psi_T.  No atomics:
 * the result is bitwise reproducible.  With the environment variable
 * MPDATA_ADJOINT=march the antidiffusive-velocity adjoint of a limited pass
 * runs as one k-marching kernel instead of two gather kernels (the same
 * result bit for bit; slower on MI355X, kept for comparison).  ws: at least the MPDATA_OP_ADJOINT
 * size for the same nsteps and checkpoint_every.  No output (dJ_dpsi0,
 * dJ_dc*, psiT_out) may alias an input, another output or the workspace
 * (MPDATA_EINVAL).  The MPDATA iterations and
 * limiter this differentiates are those of mpdata_step (paper, Section 5,
 * and the scheme's literature); the paper itself has no adjoint. */
int mpdata_adjoint(const mpdata_problem* p, int32_t nsteps, int32_t checkpoint_every,
                   const void* psi0, const void* cx, const void* cy, const void* cz,
                   const void* g, const void* dJ_dpsiT, void* dJ_dpsi0, void* dJ_dcx,
                   void* dJ_dcy, void* dJ_dcz, void* psiT_out, void* ws, size_t ws_bytes,
                   void* stream);

/* Batched runs: many independent problems, each with ntracers tracer fields
 * advected by the same winds and metric, all in one persistent launch per
 * pass (the fused corrective pass over a work list of (problem, tile, tracer,
 * plane) units, cut into equal ranges per workgroup).  The caller's problem
 * struct supplies bc, iters, limiter, dtype and eps for every item (its sizes
 * are ignored); each item supplies its sizes and device pointers.  psi holds
 * the item's ntracers fields consecutively ([tracer][nz][ny][nx]); cz may be
 * NULL.  Items must not share psi storage.  Flags:
 *   MPDATA_BATCH_GRAPH  capture the nsteps steps into a HIP graph on first
 *                       use and replay it (cached per item pointers, sizes,
 *                       nsteps, workspace, kernel variant and device);
 *   MPDATA_BATCH_TUNE   pick the kernel variant by timing one step of each
 *                       on this batch (FP32: tile rows of 32, 64 or 16 lanes,
 *                       i.e. 28 x 20, 60 x 8 or 12 x 44 interior cells per
 *                       768-thread tile, times one or two workgroups per CU,
 *                       or 1024-thread tiles (28 x 28, 60 x 12, 12 x 60
 *                       interior cells) one per CU, times the donor-cell
 *                       pass inside the first corrective pass or as its own
 *                       kernel: variants 0 .. 5 = (32, 1), (32, 2), (64, 1),
 *                       (64, 2), (16, 1), (16, 2) folded and 6 .. 11 the same
 *                       split, 12 .. 14 = 1024 threads with 32, 64, 16 lanes
 *                       folded and 15 .. 17 the same split; FP64: 0 folded,
 *                       1 split, 64 lanes, one workgroup); the
 *                       choice is kept per batch shape and appended to the
 *                       file named by the environment variable
 *                       MPDATA_TUNE_CACHE as a line "<batch shape>\t<variant>"
 *                       (a different file name is read afresh).  Tuning
 *                       synchronises `stream`; a tuning step reads the
 *                       caller's fields and writes only the workspace.
 * Without a tuned choice the variant is 0.  The environment variable
 * MPDATA_BATCH_VARIANT forces a variant (an index outside the dtype's
 * variants is MPDATA_EINVAL).
 * ws: at least mpdata_batch_workspace_bytes() for the same items.  The
 * paper's fusion and caching of the flux stages (Section 6.1, Table 2,
 * Listing 9) is what the fused pass applies; batching is this library's. */
typedef struct {
    int32_t nx, ny, nz;   /* cells, each >= 1                                    */
    int32_t ntracers;     /* >= 1                                                */
    const void* cx;       /* face Courant numbers and metric, [nz][ny][nx]       */
    const void* cy;
    const void* cz;       /* may be NULL                                         */
    const void* g;
    void* psi;            /* ntracers consecutive fields, in/out                 */
} mpdata_batch_item;

enum { MPDATA_BATCH_GRAPH = 1, MPDATA_BATCH_TUNE = 2 };

size_t mpdata_batch_workspace_bytes(const mpdata_problem* common, int32_t nitems,
                                    const mpdata_batch_item* items);
int mpdata_run_batched(const mpdata_problem* common, int32_t nitems,
                       const mpdata_batch_item* items, int32_t nsteps, int32_t flags,
                       void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Unstructured (edge-based) donor-cell step: the paper's own MPDATA dwarf
 * (Section 5): the upwind flux on every edge (Listings 4-5), the vertical
 * upwind flux with the boundary factor pivbz (Listing 7: the flux through
 * the bottom and top of a column is pivbz times the nearest interior
 * interface flux, 0 closes the column), the flux divergence at the nodes
 * over the dual volumes (Listing 8) and the update:
 *   div[n][k] = (sum over n's edges of sign * flux[e][k]) / vol[n]
 *               + (fz[n][k+1] - fz[n][k]),   out[n][k] = psi[n][k] - div / rho[n][k]
 * with flux[e][k] = max(0, vn) psi[ip1][k] + min(0, vn) psi[ip2][k].
 *
 * Layout (device arrays): per-node fields (n_nodes, nz) and per-edge fields
 * (n_edges, nz), level fastest, of the mesh's dtype.  w[n][k] (k >= 1) is
 * the vertical Courant number at the interface between levels k-1 and k;
 * w may be NULL (no vertical wind).  A positive vn[e][k] carries psi from
 * ip1 to ip2.  The connectivity is read as given: every index must be in
 * range (the library does not scan device memory; an index out of range is
 * a memory fault).  Dual volumes and rho must be positive.  The caller owns
 * every buffer; the calls enqueue on `stream` and allocate nothing. */
typedef struct {
    int32_t n_nodes, n_edges, nz;  /* >= 1, >= 0, >= 1                                 */
    int32_t dtype;                 /* MPDATA_F64 or MPDATA_F32 (fields, dual volumes)  */
    double pivbz;                  /* vertical boundary factor                         */
    const int32_t* edge_nodes;     /* (n_edges, 2): ip1, ip2                           */
    const int32_t* node_ptr;       /* (n_nodes + 1) offsets into node_edges, [0] = 0    */
    const int32_t* node_edges;     /* node n's edges at [node_ptr[n], node_ptr[n+1])   */
    const int8_t* node_sign;       /* +1 where the node is the edge's ip1, -1 for ip2  */
    const void* dual_volume;       /* (n_nodes)                                        */
} mpdata_umesh;

/* One step: psi_out must not alias psi_in. */
int mpdata_ustep(const mpdata_umesh* m, const void* psi_in, void* psi_out, const void* vn, const void* w,
                 const void* rho, void* stream);
/* nsteps steps in place on psi; ws: at least mpdata_uworkspace_bytes(m). */
size_t mpdata_uworkspace_bytes(const mpdata_umesh* m);
int mpdata_urun(const mpdata_umesh* m, int32_t nsteps, void* psi, const void* vn, const void* w,
                const void* rho, void* ws, size_t ws_bytes, void* stream);

/* Mass sum(G * psi) accumulated in FP64 (compensated) for either dtype,
 * written to *host_out.  Synchronises `stream`.  ws: at least the
 * MPDATA_OP_MASS size. */
int mpdata_mass(const mpdata_problem* p, const void* psi, const void* g,
                double* host_out, void* ws, size_t ws_bytes, void* stream);

/* Text of the last error on this thread ("" if none). */
const char* mpdata_last_error(void);

/* Kernel timing (diagnostics).  mpdata_timing_enable(1) clears the record and
 * from then on brackets every launch of the library's kernels with HIP events
 * on the launch stream; mpdata_timing_enable(0) stops recording and keeps
 * the record.
 * mpdata_timing_read() waits for the recorded events of one kernel kind and
 * returns the summed elapsed milliseconds and the number of launches.  Kinds:
 *   MPDATA_KERNEL_PASS        the fused corrective-pass kernel (passes 3 ..)
 *   MPDATA_KERNEL_DONOR       a separate donor-cell pass (one-pass steps,
 *                             MPDATA_KERNELS=split, batched runs)
 *   MPDATA_KERNEL_STAGE       the per-stage kernels (MPDATA_KERNELS=stages)
 *   MPDATA_KERNEL_USTEP       the unstructured step kernel
 *   MPDATA_KERNEL_PASS_DONOR  the first corrective pass with the donor-cell
 *                             pass folded in */
enum { MPDATA_KERNEL_PASS = 0, MPDATA_KERNEL_DONOR = 1, MPDATA_KERNEL_STAGE = 2, MPDATA_KERNEL_USTEP = 3,
       MPDATA_KERNEL_PASS_DONOR = 4 };
int mpdata_timing_enable(int32_t on);
int mpdata_timing_read(int32_t kind, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
