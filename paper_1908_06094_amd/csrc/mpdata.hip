// mpdata.hip -- the C ABI of libmpdata.so (declared in include/mpdata.h).
//
// Argument validation, workspace layout, the per-step pass driver and the
// FP64 compensated mass reduction.  Every step of the scheme runs in the HIP
// kernels of stages.hpp / fused.hpp; the host only validates and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "mpdata.h"
#include "common.hpp"
#include "stages.hpp"
#include "fused.hpp"
#include "donor.hpp"
#include "adjoint.hpp"
#include "adjoint_march.hpp"
#include "batched.hpp"
#include "unstructured.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return MPDATA_OK;
}

constexpr long long kMaxCells = 1LL << 34;   // 17 G cells: far beyond one GPU's HBM in FP32
constexpr int kMaxIters = 8;
constexpr double kEpsMin = 1e-30, kEpsMax = 1e-3;
// Input ranges the kernels are exact within (checked under MPDATA_DEBUG):
// psi in [0, kPsiMax], G in [kGMin, kGMax].  In FP64 the largest product the
// fused pass forms is G_sum * (2 psi + eps)^3 <= 2e6 * 8e300, below the
// FP64 maximum; in FP32 pair sums of psi stay below the FP32 maximum.
constexpr double kPsiMax64 = 1e100, kPsiMax32 = 1e30;
constexpr double kGMin = 1e-6, kGMax = 1e6;

int validate(const mpdata_problem* p)
{
    if (!p) return fail(MPDATA_EINVAL, "problem pointer is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(MPDATA_EINVAL, "sizes must be >= 1 (got nx=%d ny=%d nz=%d)", p->nx, p->ny, p->nz);
    if ((long long)p->nx * p->ny * p->nz > kMaxCells)
        return fail(MPDATA_EINVAL, "grid of %lld cells exceeds the supported maximum",
                    (long long)p->nx * p->ny * p->nz);
    if ((long long)p->nx * p->ny > (1LL << 30))
        return fail(MPDATA_EINVAL, "a plane of %lld cells exceeds the supported 2^30", (long long)p->nx * p->ny);
    if (p->nz > 65535 || p->ny > 65535 * 4)
        return fail(MPDATA_EINVAL, "ny=%d / nz=%d exceed the launch grid limits (ny <= 262140, nz <= 65535)",
                    p->ny, p->nz);
    for (int a = 0; a < 3; ++a)
        if (p->bc[a] != MPDATA_PERIODIC && p->bc[a] != MPDATA_CLOSED)
            return fail(MPDATA_EINVAL, "bc[%d]=%d is neither MPDATA_PERIODIC nor MPDATA_CLOSED", a, p->bc[a]);
    if (p->iters < 1 || p->iters > kMaxIters)
        return fail(MPDATA_EINVAL, "iters=%d outside [1, %d]", p->iters, kMaxIters);
    if (p->limiter != 0 && p->limiter != 1) return fail(MPDATA_EINVAL, "limiter=%d is not 0 or 1", p->limiter);
    if (p->dtype != MPDATA_F64 && p->dtype != MPDATA_F32)
        return fail(MPDATA_EINVAL, "dtype=%d is neither MPDATA_F64 nor MPDATA_F32", p->dtype);
    if (p->reserved != 0) return fail(MPDATA_EINVAL, "reserved field must be 0");
    // eps = 0 selects the default; otherwise [kEpsMin, kEpsMax].  The floor
    // keeps every guarded denominator a normal number in both precisions:
    // the FP64 pass divides once over G_sum * d0 * d1 * d2 with each d >= eps
    // (>= 2e-90 * G_min at the floor), beta over (in + eps)(out + eps), and
    // FP32 takes eps as a float.
    if (!(p->eps == 0.0 || (p->eps >= kEpsMin && p->eps <= kEpsMax)))
        return fail(MPDATA_EINVAL, "eps=%g is neither 0 (the default) nor in [%g, %g]", p->eps, kEpsMin, kEpsMax);
    return MPDATA_OK;
}

size_t elem_size(const mpdata_problem* p) { return p->dtype == MPDATA_F64 ? 8 : 4; }
long long cells(const mpdata_problem* p) { return (long long)p->nx * p->ny * p->nz; }

// Elements of an inter-pass velocity field of the fused path.
long long tiled_cells(const mpdata_problem* p)
{
    if (p->dtype == MPDATA_F64) return mpdata::fused::vel_elems<double>(p->nx, p->ny, p->nz);
    return mpdata::fused::vel_elems<float>(p->nx, p->ny, p->nz);
}

// Every workspace field starts on a 256-byte boundary and can hold a field
// in either layout.
size_t field_bytes(const mpdata_problem* p)
{
    size_t b = (size_t)std::max(cells(p), tiled_cells(p)) * elem_size(p);
    return (b + 255) & ~(size_t)255;
}

constexpr int kMassBlocks = 1024;
constexpr int kMassThreads = 256;
constexpr size_t kMassBytes = (size_t)(kMassBlocks + 1) * 2 * sizeof(double);

// Workspace of one step: two iterates, two velocity triples, two beta fields.
constexpr int kStepFields = 10;

size_t step_bytes(const mpdata_problem* p) { return kStepFields * field_bytes(p); }

mpdata::Geo geo_of(const mpdata_problem* p)
{
    mpdata::Geo g;
    g.nx = p->nx;
    g.ny = p->ny;
    g.nz = p->nz;
    g.closed_x = p->bc[0] == MPDATA_CLOSED;
    g.closed_y = p->bc[1] == MPDATA_CLOSED;
    g.closed_z = p->bc[2] == MPDATA_CLOSED;
    g.sy = p->nx;
    g.sz = (long long)p->nx * p->ny;
    return g;
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

int check_ptr(const void* ptr, const char* name, const mpdata_problem* p)
{
    if (!ptr) return fail(MPDATA_EINVAL, "%s is NULL", name);
    if (!aligned(ptr, elem_size(p))) return fail(MPDATA_EINVAL, "%s is not aligned to its element size", name);
    return MPDATA_OK;
}

int launch_status(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MPDATA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return MPDATA_OK;
}

// ---------------------------------------------------------------------------
// MPDATA_DEBUG (environment variable, any value but "0"): the calls scan
// their input tracer and metric on the device and refuse values outside the
// documented ranges (psi in [0, psi_max], G in [kGMin, kGMax], NaN in either)
// with MPDATA_EINVAL.  The scan synchronises the stream, so it is skipped
// while the stream is being captured into a graph.
// ---------------------------------------------------------------------------

bool debug_on()
{
    const char* e = getenv("MPDATA_DEBUG");
    return e && *e && strcmp(e, "0") != 0;
}

// flag = 1 where any of the n values lies outside [lo, hi] or is NaN (every
// writer stores the same value, so the unordered stores are benign)
template <class T>
__global__ void __launch_bounds__(256) k_range_check(const T* __restrict__ a, long long n, double lo, double hi,
                                                     unsigned* __restrict__ flag)
{
    bool bad = false;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const double x = (double)a[q];
        bad |= !(x >= lo && x <= hi);
    }
    if (bad) *flag = 1u;
}

// Scans `count` tracer fields of n cells each at psi (consecutive) and the
// metric g; flag: 8 bytes of device scratch.
int debug_check(int dtype, long long n, int count, const void* psi, const void* g, void* flag, hipStream_t st,
                const char* who)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return MPDATA_OK;
    unsigned* f = (unsigned*)flag;
    const double psi_max = dtype == MPDATA_F64 ? kPsiMax64 : kPsiMax32;
    mpdata::k_fill<unsigned><<<1, 64, 0, st>>>(f, 2, 0u);
    const long long np = n * count;
    if (dtype == MPDATA_F64) {
        k_range_check<double><<<1024, 256, 0, st>>>((const double*)psi, np, 0.0, psi_max, f);
        k_range_check<double><<<1024, 256, 0, st>>>((const double*)g, n, kGMin, kGMax, f + 1);
    } else {
        k_range_check<float><<<1024, 256, 0, st>>>((const float*)psi, np, 0.0, psi_max, f);
        k_range_check<float><<<1024, 256, 0, st>>>((const float*)g, n, kGMin, kGMax, f + 1);
    }
    if (int rc = launch_status("MPDATA_DEBUG range check")) return rc;
    unsigned h[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(h, f, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(MPDATA_EDEVICE, "MPDATA_DEBUG range check: %s", hipGetErrorString(e));
    if (h[0])
        return fail(MPDATA_EINVAL, "MPDATA_DEBUG: %s: psi holds values outside [0, %g] or NaN", who, psi_max);
    if (h[1]) return fail(MPDATA_EINVAL, "MPDATA_DEBUG: %s: g holds values outside [%g, %g] or NaN", who, kGMin, kGMax);
    return MPDATA_OK;
}

// ---------------------------------------------------------------------------
// Kernel timing (diagnostics): when enabled, HIP events are recorded on the
// launch stream around every kernel of a kind; reading sums their spans.
// ---------------------------------------------------------------------------

struct KernelTiming {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spans[5];
    std::vector<hipEvent_t> spare;
};
KernelTiming g_timing;

hipEvent_t timing_event()
{
    hipEvent_t e = nullptr;
    if (!g_timing.spare.empty()) {
        e = g_timing.spare.back();
        g_timing.spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// Brackets one launch of `kind` on stream `st` with events (no-op when off).
struct Timed {
    int kind;
    hipStream_t st;
    hipEvent_t e0 = nullptr;
    Timed(int k, hipStream_t s) : kind(k), st(s)
    {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        if (!g_timing.on) return;
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
        if ((e0 = timing_event()) && hipEventRecord(e0, st) != hipSuccess) e0 = nullptr;
    }
    ~Timed()
    {
        if (!e0) return;
        std::lock_guard<std::mutex> lk(g_timing.mu);
        hipEvent_t e1 = timing_event();
        if (e1 && hipEventRecord(e1, st) == hipSuccess) g_timing.spans[kind].push_back({e0, e1});
    }
};

// ---------------------------------------------------------------------------
// The pass driver (stage kernels)
// ---------------------------------------------------------------------------

template <class T>
struct StepBufs {
    T* phi[2];
    T* vel[2][3];
    T* bup;
    T* bdn;
};

template <class T>
StepBufs<T> carve(const mpdata_problem* p, void* ws)
{
    StepBufs<T> b;
    char* base = (char*)ws;
    size_t f = field_bytes(p);
    int n = 0;
    b.phi[0] = (T*)(base + f * n++);
    b.phi[1] = (T*)(base + f * n++);
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < 3; ++a) b.vel[s][a] = (T*)(base + f * n++);
    b.bup = (T*)(base + f * n++);
    b.bdn = (T*)(base + f * n++);
    return b;
}

template <class T>
int step_stages(const mpdata_problem* p, const T* psin, T* psout, const T* cx, const T* cy, const T* cz,
                const T* gm, void* ws, hipStream_t st)
{
    mpdata::Geo g = geo_of(p);
    StepBufs<T> b = carve<T>(p, ws);
    const T eps = (T)(p->eps > 0.0 ? p->eps : 1e-15);
    const double eps_d = p->eps > 0.0 ? p->eps : 1e-15;
    if (!cz) {
        // the second velocity triple's w slot is free in pass 1: zero it
        // (a fill kernel, not a memset node, so the step can be graph-captured)
        mpdata::k_fill<T><<<1024, 256, 0, st>>>(b.vel[1][2], cells(p), T(0));
        if (int rc = launch_status("zero vertical velocity")) return rc;
        cz = b.vel[1][2];
    }
    dim3 blk(64, 4, 1);
    dim3 grd((p->nx + 63) / 64, (p->ny + 3) / 4, p->nz);

    T* first_out = p->iters == 1 ? psout : b.phi[0];
    {
        Timed tm(MPDATA_KERNEL_STAGE, st);
        mpdata::stages::k_donor<T><<<grd, blk, 0, st>>>(g, psin, cx, cy, cz, gm, first_out);
    }
    if (int rc = launch_status("donor-cell pass")) return rc;
    if (p->iters == 1) return ok();

    Timed tm(MPDATA_KERNEL_STAGE, st);   // the corrective passes' stage kernels as one span
    const T* prev[3] = {cx, cy, cz};
    const T* phi = b.phi[0];
    int vsel = 0;
    for (int m = 2; m <= p->iters; ++m) {
        T* nxt = (m == p->iters) ? psout : (phi == b.phi[0] ? b.phi[1] : b.phi[0]);
        T** vq = b.vel[vsel];   // pass 2 writes triple 0, so a zeroed cz in triple 1 survives it
        mpdata::stages::k_antidiff<T><<<grd, blk, 0, st>>>(g, eps, phi, prev[0], prev[1], prev[2], gm,
                                                          vq[0], vq[1], vq[2]);
        if (int rc = launch_status("antidiffusive velocities")) return rc;
        if (p->limiter) {
            mpdata::stages::k_beta<T><<<grd, blk, 0, st>>>(g, eps_d, psin, phi, vq[0], vq[1], vq[2], gm,
                                                          b.bup, b.bdn);
            if (int rc = launch_status("limiter coefficients")) return rc;
            mpdata::stages::k_limit<T><<<grd, blk, 0, st>>>(g, vq[0], vq[1], vq[2], vq[0], vq[1], vq[2], b.bup,
                                                           b.bdn);
            if (int rc = launch_status("limited velocities")) return rc;
        }
        mpdata::stages::k_donor<T><<<grd, blk, 0, st>>>(g, phi, vq[0], vq[1], vq[2], gm, nxt);
        if (int rc = launch_status("corrective pass")) return rc;
        prev[0] = vq[0];
        prev[1] = vq[1];
        prev[2] = vq[2];
        phi = nxt;
        vsel ^= 1;
    }
    return ok();
}

// ---------------------------------------------------------------------------
// The fused driver: donor-cell pass, then one k-marching kernel per
// corrective pass.
// ---------------------------------------------------------------------------

// Compute units of the current device (cached per device).
int cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

// Persistent grid of the fused passes: one workgroup per CU (their LDS
// allows no more), a multiple of 8 (the XCD count the work split groups by),
// and no more workgroups than leave each at least ~12 output planes, except
// that a small problem spreads over up to 64 workgroups (a 64 x 64 plane has
// 16 tile planes: one workgroup each instead of 8 with two tiles in turn).
int pass_grid(long long total_planes)
{
    long long n = cu_count();
    long long cap = total_planes / 12;
    if (cap < 64) cap = total_planes < 64 ? total_planes : 64;
    if (n > cap) n = cap;
    n &= ~7LL;
    return n < 8 ? 8 : (int)n;
}

template <class T, bool LIMIT, bool WRITE_VEL, bool REC = false, bool DONOR = false>
int launch_pass(const mpdata_problem* p, const mpdata::fused::PassArgs<T>& a, hipStream_t st)
{
    mpdata::Geo g = geo_of(p);
    const long long total = (long long)a.tiles_x * a.tiles_y * p->nz;
    Timed tm(DONOR ? MPDATA_KERNEL_PASS_DONOR : MPDATA_KERNEL_PASS, st);
    using TL = typename mpdata::fused::PassThreads<T, DONOR>::TL;
    const int grid = pass_grid(total) * (DONOR ? TL::donor_wgs_per_cu : TL::wgs_per_cu);
    constexpr int threads = mpdata::fused::PassThreads<T, DONOR>::value;
    mpdata::fused::k_pass<T, LIMIT, WRITE_VEL, REC, DONOR><<<grid, threads, 0, st>>>(g, a);
    return launch_status(DONOR ? "fused donor-cell and first corrective pass" : "fused corrective pass");
}

// The first corrective pass with the donor-cell pass folded in (DONOR), or
// a plain corrective pass.
template <class T>
int launch_corrective(const mpdata_problem* p, const mpdata::fused::PassArgs<T>& a, bool last, bool donor,
                      hipStream_t st)
{
    if (donor) {
        if (p->limiter)
            return last ? launch_pass<T, true, false, false, true>(p, a, st)
                        : launch_pass<T, true, true, false, true>(p, a, st);
        return last ? launch_pass<T, false, false, false, true>(p, a, st)
                    : launch_pass<T, false, true, false, true>(p, a, st);
    }
    if (p->limiter) return last ? launch_pass<T, true, false>(p, a, st) : launch_pass<T, true, true>(p, a, st);
    return last ? launch_pass<T, false, false>(p, a, st) : launch_pass<T, false, true>(p, a, st);
}

// MPDATA_KERNELS=split: the donor-cell pass as its own kernel ahead of the
// corrective passes (the layout before the donor-cell pass was folded into
// the first corrective pass; kept as a second fused path for comparison).
bool use_split_donor()
{
    const char* e = getenv("MPDATA_KERNELS");
    return e && strcmp(e, "split") == 0;
}

template <class T>
int step_fused(const mpdata_problem* p, const T* psin, T* psout, const T* cx, const T* cy, const T* cz,
               const T* gm, void* ws, hipStream_t st)
{
    mpdata::Geo g = geo_of(p);
    StepBufs<T> b = carve<T>(p, ws);
    dim3 blk(64, 4, 1);
    // the donor-cell pass runs inside the first corrective pass, unless it is
    // the only pass (or the split layout is asked for)
    const bool fold = p->iters >= 2 && !use_split_donor();
    T* first_out = p->iters == 1 ? psout : b.phi[0];
    if (!fold) {
        Timed tm(MPDATA_KERNEL_DONOR, st);
        dim3 dgrd((p->nx + 63) / 64, (p->ny + 3) / 4, (p->nz + mpdata::fused::kDonorChunk - 1) / mpdata::fused::kDonorChunk);
        mpdata::fused::k_donor_march<T><<<dgrd, blk, 0, st>>>(g, psin, cx, cy, cz, gm, first_out);
        if (int rc = launch_status("donor-cell pass")) return rc;
    }

    mpdata::fused::PassArgs<T> a{};
    a.psin = psin;
    a.g = gm;
    a.eps = p->eps > 0.0 ? p->eps : 1e-15;
    a.tiles_x = (p->nx + mpdata::fused::Tile<T>::tile_x - 1) / mpdata::fused::Tile<T>::tile_x;
    a.tiles_y = (p->ny + mpdata::fused::Tile<T>::tile_y - 1) / mpdata::fused::Tile<T>::tile_y;
    a.u = cx;
    a.v = cy;
    a.w = cz;
    a.vel_tiled = 0;
    const T* phi = b.phi[0];
    int vsel = 0;
    for (int m = 2; m <= p->iters; ++m) {
        const bool last = m == p->iters;
        T* nxt = last ? psout : (phi == b.phi[0] ? b.phi[1] : b.phi[0]);
        const bool donor = fold && m == 2;
        a.phi = donor ? nullptr : phi;   // the donor-fused pass forms psi^(1) itself
        using DT = mpdata::fused::Tile<T, mpdata::fused::DefaultLanes<T>::value,
                                       mpdata::fused::PassThreads<T, true>::value>;   // the donor-fused pass's tile
        a.tiles_x = (p->nx + (donor ? DT::donor_tile_x : mpdata::fused::Tile<T>::tile_x) - 1) /
                    (donor ? DT::donor_tile_x : mpdata::fused::Tile<T>::tile_x);
        using PT = typename mpdata::fused::PassThreads<T, false>::TL;   // the plain pass's tile
        a.tiles_y = (p->ny + (donor ? DT::tile_y : PT::tile_y) - 1) / (donor ? DT::tile_y : PT::tile_y);
        a.out = nxt;
        a.ul = b.vel[vsel][0];
        a.vl = b.vel[vsel][1];
        a.wl = b.vel[vsel][2];
        if (int rc = launch_corrective<T>(p, a, last, donor, st)) return rc;
        a.u = a.ul;
        a.v = a.vl;
        a.w = a.wl;
        a.vel_tiled = mpdata::fused::Tile<T>::tiled_velocities;
        phi = nxt;
        vsel ^= 1;
    }
    return ok();
}

bool use_stage_kernels()
{
    const char* e = getenv("MPDATA_KERNELS");
    return e && strcmp(e, "stages") == 0;
}

// ws_bytes: the size of the region at ws (checked against what the step carves)
int dispatch_step(const mpdata_problem* p, const void* psin, void* psout, const void* cx, const void* cy,
                  const void* cz, const void* gm, void* ws, size_t ws_bytes, hipStream_t st)
{
    if (ws_bytes < step_bytes(p))
        return fail(MPDATA_EINVAL, "internal: step workspace of %zu bytes is below %zu", ws_bytes, step_bytes(p));
    const bool stages = use_stage_kernels();
    if (p->dtype == MPDATA_F64) {
        auto f = stages ? step_stages<double> : step_fused<double>;
        return f(p, (const double*)psin, (double*)psout, (const double*)cx, (const double*)cy, (const double*)cz,
                 (const double*)gm, ws, st);
    }
    auto f = stages ? step_stages<float> : step_fused<float>;
    return f(p, (const float*)psin, (float*)psout, (const float*)cx, (const float*)cy, (const float*)cz,
             (const float*)gm, ws, st);
}

// ---------------------------------------------------------------------------
// Mass: per-thread Neumaier sums in FP64, combined pairwise with an exact
// two-sum, in a fixed order (deterministic).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void two_sum_acc(double& s, double& c, double x)
{
    double t = s + x;
    double bp = t - s;
    double e = (s - (t - bp)) + (x - bp);
    s = t;
    c += e;
}

template <class T>
__global__ void __launch_bounds__(kMassThreads) k_mass_partial(long long n, const T* __restrict__ psi,
                                                               const T* __restrict__ gm, double* __restrict__ part)
{
    __shared__ double ss[kMassThreads], sc[kMassThreads];
    double s = 0.0, c = 0.0;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        two_sum_acc(s, c, (double)gm[q] * (double)psi[q]);
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int h = kMassThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            double s2 = ss[threadIdx.x], c2 = sc[threadIdx.x] + sc[threadIdx.x + h];
            two_sum_acc(s2, c2, ss[threadIdx.x + h]);
            ss[threadIdx.x] = s2;
            sc[threadIdx.x] = c2;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss[0];
        part[2 * blockIdx.x + 1] = sc[0];
    }
}

__global__ void __launch_bounds__(kMassThreads) k_mass_final(int nparts, double* __restrict__ part)
{
    __shared__ double ss[kMassThreads], sc[kMassThreads];
    double s = 0.0, c = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
        two_sum_acc(s, c, part[2 * b]);
        c += part[2 * b + 1];
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int h = kMassThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            double s2 = ss[threadIdx.x], c2 = sc[threadIdx.x] + sc[threadIdx.x + h];
            two_sum_acc(s2, c2, ss[threadIdx.x + h]);
            ss[threadIdx.x] = s2;
            sc[threadIdx.x] = c2;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[2 * nparts] = ss[0] + sc[0];
}

// ---------------------------------------------------------------------------
// Adjoint driver (FP64)
// ---------------------------------------------------------------------------

struct AdjLayout {
    long long n;          // cells
    size_t fb;            // bytes per field
    int segs, K;          // checkpoints, steps per segment
    int M;                // passes per step
    size_t fields;        // total fields
};

AdjLayout adj_layout(const mpdata_problem* p, int nsteps, int K)
{
    AdjLayout L;
    L.n = cells(p);
    L.fb = field_bytes(p);   // every field, the forward step's included, fits either layout
    L.K = K;
    L.segs = nsteps > 0 ? (nsteps + K - 1) / K : 1;
    L.M = p->iters;
    // checkpoints + segment states + for each step of a segment and each
    // corrective pass a record (the pass's input iterate, U~ x3, V x3, beta
    // x2) + the extremal-entry codes of the bounds of the step being
    // reversed, per pass + a sink for the segment's last output + 16 adjoint
    // fields (cur, prev, psin, V x3, Vprev x3, U~ x3, lin, lout, lmx, lmn) +
    // antidiffusive slots (3 axes x kSlots) + a zero field and a dJ/dcz scratch
    L.fields = (size_t)L.segs + (size_t)K + (size_t)K * 9 * (L.M - 1) + (size_t)(L.M - 1) + 1 + 16 +
               (size_t)3 * mpdata::adj::kSlots + 2;
    return L;
}

// The intermediates of one forward step that its adjoint reads, per
// corrective pass m = 2..M: phis[m - 1] (the pass's input iterate), ut / vl
// [3 m + axis] (its antidiffusive and limited velocities), bu / bd [m]
// (beta, at most 1).
struct AdjRec {
    std::vector<double*> phis, ut, vl, bu, bd;
};

// One forward step of the adjoint's sweeps, through the kernels of the
// forward path: the first corrective pass carries the donor-cell pass (a
// one-pass step is the donor-cell kernel alone), the passes hand on their
// limited velocities.  With `record` the passes are the recording variants,
// which also store psi^(1), each pass's antidiffusive velocities and beta:
// the step's intermediates land in R.  The recording and the plain variants
// evaluate the same arithmetic (they differ in stores only), so a state is
// the same whatever steps were recorded and whatever the checkpoint
// interval (tested bitwise).
int step_adjoint_fwd(const mpdata_problem* p, const double* psin, double* psout, const double* cx, const double* cy,
                     const double* cz, const double* gm, const AdjRec& R, bool record, hipStream_t st)
{
    namespace F = mpdata::fused;
    const int M = p->iters;
    if (M == 1) {
        mpdata::Geo g = geo_of(p);
        dim3 blk(64, 4, 1);
        dim3 dgrd((p->nx + 63) / 64, (p->ny + 3) / 4, (p->nz + F::kDonorChunk - 1) / F::kDonorChunk);
        F::k_donor_march<double><<<dgrd, blk, 0, st>>>(g, psin, cx, cy, cz, gm, psout);
        return launch_status("adjoint: donor-cell pass");
    }
    F::PassArgs<double> a{};
    a.psin = psin;
    a.g = gm;
    a.eps = p->eps > 0.0 ? p->eps : 1e-15;
    a.vel_tiled = 0;
    using DT = F::PassThreads<double, true>::TL;    // the donor-fused pass's tile
    using PT = F::PassThreads<double, false>::TL;   // the plain pass's
    for (int m = 2; m <= M; ++m) {
        const bool donor = m == 2, last = m == M;
        const int tile_x = donor ? DT::donor_tile_x : PT::tile_x;
        const int tile_y = donor ? DT::tile_y : PT::tile_y;
        a.tiles_x = (p->nx + tile_x - 1) / tile_x;
        a.tiles_y = (p->ny + tile_y - 1) / tile_y;
        a.phi = donor ? nullptr : R.phis[m - 1];
        a.rphi = record && donor ? R.phis[1] : nullptr;
        a.out = last ? psout : R.phis[m];
        a.u = m == 2 ? cx : R.vl[3 * (m - 1)];
        a.v = m == 2 ? cy : R.vl[3 * (m - 1) + 1];
        a.w = m == 2 ? cz : R.vl[3 * (m - 1) + 2];
        a.ul = R.vl[3 * m];
        a.vl = R.vl[3 * m + 1];
        a.wl = R.vl[3 * m + 2];
        a.rux = R.ut[3 * m];
        a.ruy = R.ut[3 * m + 1];
        a.ruz = R.ut[3 * m + 2];
        a.rbu = R.bu[m];
        a.rbd = R.bd[m];
        int rc;
        if (record) {
            if (donor)
                rc = p->limiter ? launch_pass<double, true, true, true, true>(p, a, st)
                                : launch_pass<double, false, true, true, true>(p, a, st);
            else
                rc = p->limiter ? launch_pass<double, true, true, true>(p, a, st)
                                : launch_pass<double, false, true, true>(p, a, st);
        } else {
            // the plain passes: the last one writes no velocities
            rc = launch_corrective<double>(p, a, last, donor, st);
        }
        if (rc) return rc;
    }
    return MPDATA_OK;
}

// MPDATA_ADJOINT=march: the antidiffusive-velocity adjoint of a limited
// pass as one k-marching kernel (adjoint_march.hpp) instead of its two
// gather kernels with the slot fields in HBM; the results are the same bit
// for bit.
bool use_adjoint_march()
{
    const char* e = getenv("MPDATA_ADJOINT");
    return e && strcmp(e, "march") == 0;
}

int adjoint_run(const mpdata_problem* p, int nsteps, int K, const double* psi0, const double* cx, const double* cy,
                const double* cz, const double* gm, const double* seed, double* dpsi0, double* dcx, double* dcy,
                double* dcz, double* psiT, void* ws, hipStream_t st)
{
    namespace A = mpdata::adj;
    const AdjLayout L = adj_layout(p, nsteps, K);
    const long long n = L.n;
    char* base = (char*)ws;
    size_t next = 0;
    auto field = [&]() { double* f = (double*)(base + L.fb * next); ++next; return f; };
    std::vector<double*> ckpt(L.segs), seg(K);
    for (auto& f : ckpt) f = field();
    for (auto& f : seg) f = field();
    const int M = L.M;
    // per-step records of a segment, and the bounds of the step being reversed
    std::vector<AdjRec> rec(K);
    for (AdjRec& R : rec) {
        R.phis.assign(M + 1, nullptr);
        R.ut.assign(3 * (M + 1), nullptr);
        R.vl.assign(3 * (M + 1), nullptr);
        R.bu.assign(M + 1, nullptr);
        R.bd.assign(M + 1, nullptr);
        for (int m = 2; m <= M; ++m) {
            R.phis[m - 1] = field();
            R.bu[m] = field();
            R.bd[m] = field();
            for (int a = 0; a < 3; ++a) {
                R.ut[3 * m + a] = field();
                R.vl[3 * m + a] = field();
            }
        }
    }
    std::vector<unsigned char*> code(M + 1, nullptr);   // 2 bytes per cell in a field of 8
    for (int m = 2; m <= M; ++m) code[m] = (unsigned char*)field();
    double* sink = field();
    double* lcur = field();
    double* lprev = field();
    double* lpsin = field();
    double* lv[3] = {field(), field(), field()};
    double* lvp[3] = {field(), field(), field()};
    double* lut[3] = {field(), field(), field()};
    double* lin = field();
    double* lout = field();
    double* lmx = field();
    double* lmn = field();
    double* slots = field();
    next += 3 * mpdata::adj::kSlots - 1;   // the slot fields are contiguous
    double* zero_w = field();
    double* dcz_scratch = field();
    const long long slot_stride = (long long)(L.fb / sizeof(double));
    if (next != L.fields)   // the carve above must match the size the caller allocated
        return fail(MPDATA_EINVAL, "internal: adjoint workspace layout mismatch (%zu != %zu fields)", next,
                    L.fields);

    mpdata::Geo g = geo_of(p);
    dim3 blk(64, 4, 1);
    dim3 grd((p->nx + 63) / 64, (p->ny + 3) / 4, p->nz);
    const double eps = p->eps > 0.0 ? p->eps : 1e-15;
    auto fill0 = [&](double* a) { mpdata::k_fill<double><<<1024, 256, 0, st>>>(a, n, 0.0); };
    hipError_t copy_err = hipSuccess;
    auto copy = [&](double* dst, const double* src) {
        hipError_t e = hipMemcpyAsync(dst, src, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (copy_err == hipSuccess) copy_err = e;
    };
    if (!cz) {
        fill0(zero_w);
        cz = zero_w;
    }
    double* dcz_t = dcz ? dcz : dcz_scratch;   // without a dcz output its sums land in scratch
    const double* C3[3] = {cx, cy, cz};
    double* dC[3] = {dcx, dcy, dcz_t};
    Timed tm(MPDATA_KERNEL_STAGE, st);
    const bool march = use_adjoint_march();

    // forward sweep: psi^{cK} into checkpoint c, other states ping-pong
    // between two scratch fields (the adjoint ones, unused until the
    // reverse).  The last segment's steps keep their records and states
    // right away, so the reverse sweep does not recompute that segment.
    copy(ckpt[0], psi0);
    const int last0 = (L.segs - 1) * K;
    const double* cur = ckpt[0];
    double* pp[2] = {lprev, lpsin};
    for (int s = 0; s < nsteps; ++s) {
        const int r = s - last0;
        double* dst;
        if (r >= 0)
            dst = s + 1 < nsteps ? seg[r + 1] : pp[0];
        else
            dst = (s + 1) % K == 0 ? ckpt[(s + 1) / K] : (cur == pp[0] ? pp[1] : pp[0]);
        // before the last segment no record is kept: the plain kernels
        if (int rc = step_adjoint_fwd(p, cur, dst, cx, cy, cz, gm, rec[r >= 0 ? r : 0], r >= 0, st)) return rc;
        cur = dst;
    }
    if (psiT && cur != psiT) copy(psiT, cur);

    copy(lcur, seed);
    for (int a = 0; a < 3; ++a) fill0(dC[a]);

    for (int sg = L.segs - 1; sg >= 0; --sg) {
        const int s0 = sg * K;
        const int s1 = (s0 + K < nsteps) ? s0 + K : nsteps;
        // step r of the segment starts from state(r)
        auto state = [&](int r) -> const double* { return r == 0 ? ckpt[sg] : seg[r]; };
        // the segment's steps again from its checkpoint, by the same kernels
        // as the forward sweep, keeping each step's intermediates (the last
        // segment's are kept from the forward sweep)
        if (sg < L.segs - 1)
            for (int r = 0; r < s1 - s0; ++r)
                if (int rc = step_adjoint_fwd(p, state(r), r + 1 < s1 - s0 ? seg[r + 1] : sink, cx, cy, cz, gm,
                                              rec[r], true, st))
                    return rc;
        for (int r = s1 - s0 - 1; r >= 0; --r) {
            const AdjRec& R = rec[r];
            const double* psin = state(r);
            // reverse through the passes.  No buffer is cleared: the first
            // contribution each adjoint buffer receives in a step assigns it.
            for (int m = M; m >= 2; --m) {
                const double* ph = R.phis[m - 1];
                const double* prev[3];
                for (int a = 0; a < 3; ++a) prev[a] = m == 2 ? C3[a] : R.vl[3 * (m - 1) + a];
                const double* U3[3] = {R.ut[3 * m], R.ut[3 * m + 1], R.ut[3 * m + 2]};
                const double* V3[3] = {R.vl[3 * m], R.vl[3 * m + 1], R.vl[3 * m + 2]};
                if (p->limiter)
                    // the donor-cell adjoint fused with the limiter's per-cell terms
                    A::k_adj_donor_limit_beta<<<grd, blk, 0, st>>>(g, eps, ph, V3[0], V3[1], V3[2], gm, lcur, lv[0],
                                                                   lv[1], lv[2], m == M, U3[0], U3[1], U3[2],
                                                                   R.bu[m], R.bd[m], psin, code[m], lut[0], lut[1],
                                                                   lut[2], lin, lout, lmx, lmn, lprev);
                else
                    A::k_adj_donor<<<grd, blk, 0, st>>>(g, ph, V3[0], V3[1], V3[2], gm, lcur, lprev, lv[0], lv[1],
                                                        lv[2], 1, m == M);
                double* tgt[3];
                for (int a = 0; a < 3; ++a) tgt[a] = m == 2 ? dC[a] : lvp[a];
                if (p->limiter && march) {
                    // the limiter's in / out and bounds gather and the
                    // antidiffusive velocities' adjoint in one k-marching
                    // kernel; the cells near closed ends are gathered after
                    A::MarchArgs ma{};
                    ma.eps = eps;
                    ma.phi = ph;
                    ma.ut = U3[0];
                    ma.vt = U3[1];
                    ma.wt = U3[2];
                    ma.lin = lin;
                    ma.lout = lout;
                    ma.lmx = lmx;
                    ma.lmn = lmn;
                    ma.code = code[m];
                    ma.lutx = lut[0];
                    ma.luty = lut[1];
                    ma.lutz = lut[2];
                    ma.pu = prev[0];
                    ma.pv = prev[1];
                    ma.pw = prev[2];
                    ma.gm = gm;
                    ma.lpsin = lpsin;
                    ma.slots = slots;
                    ma.field = slot_stride;
                    ma.lphi = lprev;
                    ma.lu = tgt[0];
                    ma.lv = tgt[1];
                    ma.lw = tgt[2];
                    ma.assign_psin = m == M;
                    ma.assign_vel = m > 2;
                    ma.tiles_x = (p->nx + A::kMTileX - 1) / A::kMTileX;
                    ma.tiles_y = (p->ny + A::kMTileY - 1) / A::kMTileY;
                    const int mgrid = pass_grid((long long)ma.tiles_x * ma.tiles_y * p->nz);
                    A::k_adj_antidiff_march<<<mgrid, A::kMThreads, 0, st>>>(g, ma);
                    A::k_adj_antidiff2<<<grd, blk, 0, st>>>(g, slots, slot_stride, lprev, tgt[0], tgt[1], tgt[2], 1);
                } else {
                    if (p->limiter)
                        // the limiter's in / out and bounds gather fused with the
                        // antidiffusive velocities' first adjoint kernel
                        A::k_adj_inout_bounds_antidiff1<<<grd, blk, 0, st>>>(
                            g, eps, ph, U3[0], U3[1], U3[2], lin, lout, code[m], lmx, lmn, lut[0], lut[1], lut[2],
                            lpsin, m == M, prev[0], prev[1], prev[2], gm, slots, slot_stride, lprev, tgt[0], tgt[1],
                            tgt[2], m > 2);
                    else   // unlimited: dJ/dU~ = dJ/dV
                        A::k_adj_antidiff1<<<grd, blk, 0, st>>>(g, eps, ph, prev[0], prev[1], prev[2], gm, lv[0],
                                                                lv[1], lv[2], slots, slot_stride, lprev, tgt[0],
                                                                tgt[1], tgt[2], m > 2);
                    A::k_adj_antidiff2<<<grd, blk, 0, st>>>(g, slots, slot_stride, lprev, tgt[0], tgt[1], tgt[2],
                                                            0);
                }
                std::swap(lcur, lprev);
                for (int a = 0; a < 3; ++a) std::swap(lv[a], lvp[a]);
            }
            A::k_adj_donor<<<grd, blk, 0, st>>>(g, psin, cx, cy, cz, gm, lcur, lpsin, dC[0], dC[1], dC[2],
                                                !(p->limiter && M >= 2), 0);
            std::swap(lcur, lpsin);
            if (int rc = launch_status("adjoint step")) return rc;
        }
    }
    copy(dpsi0, lcur);
    if (copy_err != hipSuccess) return fail(MPDATA_EDEVICE, "adjoint copies: %s", hipGetErrorString(copy_err));
    return ok();
}

// ---------------------------------------------------------------------------
// Batched driver
// ---------------------------------------------------------------------------

int validate_items(const mpdata_problem* c, int n, const mpdata_batch_item* items)
{
    if (n < 1) return fail(MPDATA_EINVAL, "nitems=%d must be >= 1", n);
    if (!items) return fail(MPDATA_EINVAL, "items is NULL");
    const size_t el = elem_size(c);
    long long donor_blocks = 0;
    for (int i = 0; i < n; ++i) {
        const mpdata_batch_item& it = items[i];
        if (it.nx < 1 || it.ny < 1 || it.nz < 1 || it.nz > 65535 || it.ny > 65535 * 4 ||
            (long long)it.nx * it.ny > (1LL << 30))
            return fail(MPDATA_EINVAL, "item %d: sizes %dx%dx%d out of range", i, it.nx, it.ny, it.nz);
        if (it.ntracers < 1) return fail(MPDATA_EINVAL, "item %d: ntracers=%d must be >= 1", i, it.ntracers);
        const void* req[] = {it.cx, it.cy, it.g, it.psi};
        for (const void* q : req)
            if (!q || !aligned(q, el)) return fail(MPDATA_EINVAL, "item %d: a required pointer is NULL or misaligned", i);
        if (it.cz && !aligned(it.cz, el)) return fail(MPDATA_EINVAL, "item %d: cz is misaligned", i);
        donor_blocks += (long long)((it.nx + 63) / 64) * ((it.ny + 3) / 4) *
                        ((it.nz + mpdata::fused::kDonorChunk - 1) / mpdata::fused::kDonorChunk) * it.ntracers;
        if (donor_blocks > 0x7fffffffLL) return fail(MPDATA_EINVAL, "the batch exceeds 2^31-1 donor-pass blocks");
    }
    return MPDATA_OK;
}

struct BatchCacheEntry {
    hipGraphExec_t exec = nullptr;
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t upload_done = nullptr;
    int variant = -1;
};

std::mutex g_batch_mu;
std::map<std::string, BatchCacheEntry> g_batch_cache;
std::map<std::string, int> g_tuned;          // batch shape -> variant (from tuning or MPDATA_TUNE_CACHE)
std::string g_tune_path;                     // the cache file g_tuned was read from
bool g_tune_file_read = false;
hipStream_t g_capture_stream[64] = {nullptr};

// Kernel variants of the batched passes: the tile row width, the
// workgroups per CU (waves per SIMD) and whether the donor-cell pass runs
// inside the first corrective pass or as its own kernel (in FP32 the
// separate donor-cell kernel is cheap, half the bytes of FP64, and the
// folded one costs about as much in arithmetic, so which is faster depends
// on the batch).  FP32 has twelve variants, FP64 two.
struct BatchVariant {
    int lanes, waves_per_simd;
    bool fold;
    int threads;   // per workgroup: 768 (12 waves) or 1024 (16 waves, 1024 / lanes rows)
};
constexpr BatchVariant kVariantsF32[] = {
    {32, 3, true, 768},   {32, 6, true, 768},   {64, 3, true, 768},   {64, 6, true, 768},
    {16, 3, true, 768},   {16, 6, true, 768},   {32, 3, false, 768},  {32, 6, false, 768},
    {64, 3, false, 768},  {64, 6, false, 768},  {16, 3, false, 768},  {16, 6, false, 768},
    {32, 4, true, 1024},  {64, 4, true, 1024},  {16, 4, true, 1024},
    {32, 4, false, 1024}, {64, 4, false, 1024}, {16, 4, false, 1024}};
constexpr BatchVariant kVariantsF64[] = {{64, 3, true, 768}, {64, 3, false, 768}};
int variant_count(int dtype) { return dtype == MPDATA_F32 ? 18 : 2; }
BatchVariant variant_of(int dtype, int v) { return dtype == MPDATA_F32 ? kVariantsF32[v] : kVariantsF64[v]; }

std::string shape_key(const mpdata_problem* c, int n, const mpdata_batch_item* items)
{
    std::string k;
    char buf[96];
    snprintf(buf, sizeof buf, "d%d i%d l%d b%d%d%d n%d", c->dtype, c->iters, c->limiter, c->bc[0], c->bc[1], c->bc[2], n);
    k += buf;
    for (int i = 0; i < n; ++i) {
        snprintf(buf, sizeof buf, ";%dx%dx%dt%d%s", items[i].nx, items[i].ny, items[i].nz, items[i].ntracers,
                 items[i].cz ? "" : "z");
        k += buf;
    }
    return k;
}

// (Re-)reads the tuning cache named by MPDATA_TUNE_CACHE whenever that name
// differs from the one read last: the choices of one cache file never
// answer for another.
void read_tune_file()
{
    const char* path = getenv("MPDATA_TUNE_CACHE");
    const std::string now = path ? path : "";
    if (g_tune_file_read && now == g_tune_path) return;
    g_tuned.clear();
    g_tune_path = now;
    g_tune_file_read = true;
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[1 << 16];
    while (fgets(line, sizeof line, f)) {
        char* tab = strrchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        g_tuned[line] = atoi(tab + 1);
    }
    fclose(f);
}

void write_tune_file(const std::string& key, int variant)
{
    const char* path = getenv("MPDATA_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s\t%d\n", key.c_str(), variant);
    fclose(f);
}

template <class T>
struct BatchDev {
    const mpdata::fused::DonorBlocks<T>* donor[2];
    const mpdata::fused::BatchEntry<T>* pass[2][8];
    const mpdata::stages::DonorEntry<T>* copyback;
};

// One step's launches for the variant of row width LANES, WPS waves per SIMD
// and N threads per workgroup: the donor-cell pass unless the first
// corrective pass carries it, then the corrective passes.
template <class T, int LANES, int WPS, int N = mpdata::fused::kThreads>
int enqueue_batched_step_v(const mpdata_problem* c, int n, const batch::Tables<T>& tb, const BatchDev<T>& dv, int par,
                           hipStream_t st)
{
    const int cus = cu_count();
    if (!tb.fold) {
        Timed td(MPDATA_KERNEL_DONOR, st);
        mpdata::fused::k_donor_march_batched<T><<<(unsigned)tb.donor_blocks, 256, 0, st>>>(dv.donor[par], n);
        if (int rc = launch_status("batched donor-cell pass")) return rc;
    }
    for (int m = 2; m <= c->iters; ++m) {
        const bool last = m == c->iters;
        const bool donor = tb.fold && m == 2;
        const mpdata::fused::BatchEntry<T>* tab = dv.pass[par][m - 2];
        const long long total = tb.pass_total[m - 2];
        long long g1 = std::min<long long>(cus, std::max<long long>(8, (total / 12) & ~7LL));
        g1 &= ~7LL;
        if (g1 < 8) g1 = 8;
        const int grid = (int)(WPS == 6 ? g1 * 2 : g1);
        Timed tm(donor ? MPDATA_KERNEL_PASS_DONOR : MPDATA_KERNEL_PASS, st);
#define MPDATA_LAUNCH(LIM, WV, DN) \
    mpdata::fused::k_pass_batched<T, LIM, WV, WPS, DN, LANES, N><<<grid, N, 0, st>>>(tab, n, total)
        if (donor) {
            if (c->limiter) { if (last) MPDATA_LAUNCH(true, false, true); else MPDATA_LAUNCH(true, true, true); }
            else { if (last) MPDATA_LAUNCH(false, false, true); else MPDATA_LAUNCH(false, true, true); }
        } else {
            if (c->limiter) { if (last) MPDATA_LAUNCH(true, false, false); else MPDATA_LAUNCH(true, true, false); }
            else { if (last) MPDATA_LAUNCH(false, false, false); else MPDATA_LAUNCH(false, true, false); }
        }
#undef MPDATA_LAUNCH
        if (int rc = launch_status("batched corrective pass")) return rc;
    }
    return MPDATA_OK;
}

template <class T>
int enqueue_batched_step(const mpdata_problem* c, int n, const batch::Tables<T>& tb, const BatchDev<T>& dv, int par,
                         int variant, hipStream_t st)
{
    if constexpr (sizeof(T) == 8) {
        return variant >= 0 && variant < 2 ? enqueue_batched_step_v<T, 64, 3>(c, n, tb, dv, par, st)
                                           : fail(MPDATA_EINVAL, "batched kernel variant %d does not exist in FP64",
                                                  variant);
    } else {
        // the fold is the tables' (variants v and v + 6 of the first twelve,
        // and v and v + 3 of the last six, share their kernels)
        if (variant >= 12 && variant < 18) {
            switch ((variant - 12) % 3) {
            case 0: return enqueue_batched_step_v<T, 32, 4, 1024>(c, n, tb, dv, par, st);
            case 1: return enqueue_batched_step_v<T, 64, 4, 1024>(c, n, tb, dv, par, st);
            default: return enqueue_batched_step_v<T, 16, 4, 1024>(c, n, tb, dv, par, st);
            }
        }
        switch (variant % 6) {
        case 0: return enqueue_batched_step_v<T, 32, 3>(c, n, tb, dv, par, st);
        case 1: return enqueue_batched_step_v<T, 32, 6>(c, n, tb, dv, par, st);
        case 2: return enqueue_batched_step_v<T, 64, 3>(c, n, tb, dv, par, st);
        case 3: return enqueue_batched_step_v<T, 64, 6>(c, n, tb, dv, par, st);
        case 4: return enqueue_batched_step_v<T, 16, 3>(c, n, tb, dv, par, st);
        case 5: return enqueue_batched_step_v<T, 16, 6>(c, n, tb, dv, par, st);
        default: return fail(MPDATA_EINVAL, "batched kernel variant %d does not exist", variant);
        }
    }
}

// Tables for a variant (its tile width decides the work units).
template <class T>
batch::Tables<T> tables_for(const mpdata_problem* c, int n, const mpdata_batch_item* items, const batch::Layout& L,
                            char* ws, int variant)
{
    // MPDATA_KERNELS=split keeps the donor-cell pass separate whatever the variant
    const bool fold = c->iters >= 2 && !use_split_donor() && variant_of(c->dtype, variant).fold;
    if constexpr (sizeof(T) == 8) {
        return batch::build_tables<T, 64>(c, n, items, L, ws, fold);
    } else {
        const int lanes = kVariantsF32[variant].lanes;
        if (kVariantsF32[variant].threads == 1024) {
            if (lanes == 16) return batch::build_tables<T, 16, 1024>(c, n, items, L, ws, fold);
            if (lanes == 32) return batch::build_tables<T, 32, 1024>(c, n, items, L, ws, fold);
            return batch::build_tables<T, 64, 1024>(c, n, items, L, ws, fold);
        }
        if (lanes == 16) return batch::build_tables<T, 16>(c, n, items, L, ws, fold);
        if (lanes == 32) return batch::build_tables<T, 32>(c, n, items, L, ws, fold);
        return batch::build_tables<T, 64>(c, n, items, L, ws, fold);
    }
}

template <class T>
int enqueue_batched_run(const mpdata_problem* c, int n, const batch::Tables<T>& tb, const BatchDev<T>& dv,
                        int nsteps, int variant, hipStream_t st)
{
    for (int s = 0; s < nsteps; ++s)
        if (int rc = enqueue_batched_step<T>(c, n, tb, dv, s & 1, variant, st)) return rc;
    if (nsteps & 1) {
        batch::k_copy_batched<T><<<cu_count() * 8, 256, 0, st>>>(dv.copyback, n, tb.donor_total);
        if (int rc = launch_status("batched copy-back")) return rc;
    }
    return MPDATA_OK;
}

// Host image of the tables in the workspace's table region, and the device
// addresses of each table: donor[0], donor[1], pass[0][*], pass[1][*],
// copyback, each in a slot of n entries of the largest entry type.
template <class T>
void pack_tables(const mpdata_problem* c, int n, const batch::Tables<T>& tb, void* ws, std::vector<char>& host,
                 BatchDev<T>& dv)
{
    const size_t slot = std::max(sizeof(mpdata::fused::BatchEntry<double>),
                                 std::max(sizeof(mpdata::stages::DonorEntry<double>),
                                          sizeof(mpdata::fused::DonorBlocks<double>))) * n;
    size_t off = 0;
    auto put = [&](const void* src, size_t bytes) {
        memcpy(host.data() + off, src, bytes);
        const void* dev = (const char*)ws + off;
        off += slot;
        return dev;
    };
    for (int par = 0; par < 2; ++par)
        dv.donor[par] = (const mpdata::fused::DonorBlocks<T>*)put(tb.donor[par].data(), sizeof(tb.donor[par][0]) * n);
    for (int par = 0; par < 2; ++par)
        for (int m = 2; m <= c->iters; ++m)
            dv.pass[par][m - 2] =
                (const mpdata::fused::BatchEntry<T>*)put(tb.pass[par][m - 2].data(), sizeof(tb.pass[par][0][0]) * n);
    dv.copyback = (const mpdata::stages::DonorEntry<T>*)put(tb.copyback.data(), sizeof(tb.copyback[0]) * n);
}

// MPDATA_BATCH_VARIANT (environment, read per call): force a kernel variant
// (0 .. variants - 1) instead of the tuned or default one.
int forced_variant(int dtype)
{
    const char* e = getenv("MPDATA_BATCH_VARIANT");
    if (!e || !*e) return -1;
    const int v = atoi(e);
    return v >= 0 && v < variant_count(dtype) ? v : -2;
}

template <class T>
int run_batched(const mpdata_problem* c, int n, const mpdata_batch_item* items, int nsteps, int flags, void* ws,
                hipStream_t st)
{
    const batch::Layout L = batch::layout(c, n, items);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(MPDATA_EDEVICE, "no current device");

    std::lock_guard<std::mutex> lk(g_batch_mu);
    // kernel variant: forced, tuned (per batch shape), else the default (0)
    const std::string skey = shape_key(c, n, items);
    read_tune_file();
    int variant = forced_variant(c->dtype);
    if (variant == -2)
        return fail(MPDATA_EINVAL, "MPDATA_BATCH_VARIANT names no variant of this dtype (0 .. %d)",
                    variant_count(c->dtype) - 1);
    std::vector<char> host(L.table_bytes, 0);
    if (variant < 0) {
        auto it = g_tuned.find(skey);
        if (it != g_tuned.end() && it->second >= 0 && it->second < variant_count(c->dtype)) {
            variant = it->second;
        } else if ((flags & MPDATA_BATCH_TUNE) && variant_count(c->dtype) > 1) {
            // time one step of each variant on the caller's data (a step of
            // parity 0 reads the caller's fields and writes only workspace
            // fields; tuning synchronises the stream)
            struct Events {
                hipEvent_t e[2] = {nullptr, nullptr};
                ~Events()
                {
                    for (hipEvent_t x : e)
                        if (x) (void)hipEventDestroy(x);
                }
            } ev;
            if (hipEventCreate(&ev.e[0]) != hipSuccess || hipEventCreate(&ev.e[1]) != hipSuccess)
                return fail(MPDATA_EDEVICE, "tuning events");
            float best = 1e30f;
            variant = 0;
            for (int v = 0; v < variant_count(c->dtype); ++v) {
                const batch::Tables<T> tv = tables_for<T>(c, n, items, L, (char*)ws, v);
                BatchDev<T> dvv;
                pack_tables<T>(c, n, tv, ws, host, dvv);
                if (hipStreamSynchronize(st) != hipSuccess ||
                    hipMemcpyAsync(ws, host.data(), L.table_bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess)
                    return fail(MPDATA_EDEVICE, "tuning table upload");
                float ms = 0.0f;
                for (int rep = 0; rep < 2; ++rep) {   // the first is a warm-up
                    if (hipEventRecord(ev.e[0], st) != hipSuccess) return fail(MPDATA_EDEVICE, "tuning event record");
                    if (int rc = enqueue_batched_step<T>(c, n, tv, dvv, 0, v, st)) return rc;
                    if (hipEventRecord(ev.e[1], st) != hipSuccess || hipEventSynchronize(ev.e[1]) != hipSuccess ||
                        hipEventElapsedTime(&ms, ev.e[0], ev.e[1]) != hipSuccess)
                        return fail(MPDATA_EDEVICE, "tuning run failed");
                }
                if (ms < best) {
                    best = ms;
                    variant = v;
                }
            }
            g_tuned[skey] = variant;
            write_tune_file(skey, variant);
        } else {
            variant = 0;
        }
    }

    const batch::Tables<T> tb = tables_for<T>(c, n, items, L, (char*)ws, variant);
    BatchDev<T> dv;
    pack_tables<T>(c, n, tb, ws, host, dv);

    char kb[192];
    snprintf(kb, sizeof kb, "|dev%d|ws%p|s%d|f%d|v%d|fold%d", dev, ws, nsteps, flags & MPDATA_BATCH_GRAPH, variant,
             (int)tb.fold);
    std::string key = skey + kb;
    for (int i = 0; i < n; ++i) {
        char pb[160];
        snprintf(pb, sizeof pb, "|%p,%p,%p,%p,%p", items[i].psi, items[i].cx, items[i].cy, items[i].cz, items[i].g);
        key += pb;
    }
    if (g_batch_cache.size() >= 16 && !g_batch_cache.count(key)) {
        // bounded cache: retire every entry once its last upload is done
        for (auto& kv : g_batch_cache) {
            BatchCacheEntry& old = kv.second;
            if (old.upload_done) {
                (void)hipEventSynchronize(old.upload_done);
                (void)hipEventDestroy(old.upload_done);
            }
            if (old.pinned) (void)hipHostFree(old.pinned);
            if (old.exec) (void)hipGraphExecDestroy(old.exec);
        }
        g_batch_cache.clear();
    }
    BatchCacheEntry& ce = g_batch_cache[key];
    if (!ce.pinned) {
        if (hipHostMalloc(&ce.pinned, L.table_bytes, hipHostMallocDefault) != hipSuccess)
            return fail(MPDATA_EDEVICE, "pinned staging buffer for the batch tables");
        ce.pinned_bytes = L.table_bytes;
        if (hipEventCreateWithFlags(&ce.upload_done, hipEventDisableTiming) != hipSuccess)
            return fail(MPDATA_EDEVICE, "event for the batch tables");
    } else if (hipEventSynchronize(ce.upload_done) != hipSuccess) {
        return fail(MPDATA_EDEVICE, "waiting for the previous table upload");
    }
    memcpy(ce.pinned, host.data(), L.table_bytes);
    if (hipMemcpyAsync(ws, ce.pinned, L.table_bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(ce.upload_done, st) != hipSuccess)
        return fail(MPDATA_EDEVICE, "batch table upload");
    ce.variant = variant;

    if (!(flags & MPDATA_BATCH_GRAPH)) return enqueue_batched_run<T>(c, n, tb, dv, nsteps, variant, st);

    if (!ce.exec) {
        if (!g_capture_stream[dev] && hipStreamCreateWithFlags(&g_capture_stream[dev], hipStreamNonBlocking) != hipSuccess)
            return fail(MPDATA_EDEVICE, "capture stream");
        hipStream_t cs = g_capture_stream[dev];
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(MPDATA_EDEVICE, "graph capture could not start");
        int rc = enqueue_batched_run<T>(c, n, tb, dv, nsteps, variant, cs);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess || !graph) return fail(MPDATA_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&ce.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(MPDATA_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    hipError_t e = hipGraphLaunch(ce.exec, st);
    if (e != hipSuccess) return fail(MPDATA_EDEVICE, "graph launch failed: %s", hipGetErrorString(e));
    return ok();
}

// ---------------------------------------------------------------------------
// Unstructured (edge-based) donor-cell step
// ---------------------------------------------------------------------------

size_t uelem(const mpdata_umesh* m) { return m->dtype == MPDATA_F64 ? 8 : 4; }

int validate_umesh(const mpdata_umesh* m)
{
    if (!m) return fail(MPDATA_EINVAL, "mesh pointer is NULL");
    if (m->n_nodes < 1 || m->n_edges < 0 || m->nz < 1)
        return fail(MPDATA_EINVAL, "mesh sizes n_nodes=%d n_edges=%d nz=%d out of range", m->n_nodes, m->n_edges,
                    m->nz);
    if ((long long)m->n_nodes * m->nz > (1LL << 40) || (long long)m->n_edges * m->nz > (1LL << 40))
        return fail(MPDATA_EINVAL, "mesh too large");
    if (m->dtype != MPDATA_F64 && m->dtype != MPDATA_F32)
        return fail(MPDATA_EINVAL, "dtype=%d is neither MPDATA_F64 nor MPDATA_F32", m->dtype);
    if (!std::isfinite(m->pivbz)) return fail(MPDATA_EINVAL, "pivbz is not finite");
    if (!m->node_ptr || !aligned(m->node_ptr, 4) || !m->dual_volume || !aligned(m->dual_volume, uelem(m)))
        return fail(MPDATA_EINVAL, "node_ptr or dual_volume is NULL or misaligned");
    if (m->n_edges > 0 && (!m->edge_nodes || !aligned(m->edge_nodes, 4) || !m->node_edges ||
                           !aligned(m->node_edges, 4) || !m->node_sign))
        return fail(MPDATA_EINVAL, "an edge table is NULL or misaligned");
    return MPDATA_OK;
}

int check_ufield(const void* a, const char* what, const mpdata_umesh* m)
{
    if (!a) return fail(MPDATA_EINVAL, "%s is NULL", what);
    if (!aligned(a, uelem(m))) return fail(MPDATA_EINVAL, "%s is not aligned to its element size", what);
    return MPDATA_OK;
}

template <class T>
int ustep(const mpdata_umesh* m, const void* psi, void* out, const void* vn, const void* w, const void* rho,
          hipStream_t st)
{
    mpdata::unstructured::UArgs<T> a;
    a.edge_nodes = m->edge_nodes;
    a.node_ptr = m->node_ptr;
    a.node_edges = m->node_edges;
    a.node_sign = m->node_sign;
    a.vol = (const T*)m->dual_volume;
    a.psi = (const T*)psi;
    a.vn = (const T*)vn;
    a.w = (const T*)w;
    a.rho = (const T*)rho;
    a.out = (T*)out;
    a.pivbz = (T)m->pivbz;
    a.n_nodes = m->n_nodes;
    a.nz = m->nz;
    Timed tm(MPDATA_KERNEL_USTEP, st);
    const char* mode = getenv("MPDATA_USTEP");
    const bool fits32 = (long long)m->n_nodes * m->nz < (1LL << 31) && (long long)m->n_edges * m->nz < (1LL << 31);
    if (!fits32 || (mode && strcmp(mode, "wave") == 0)) {
        const unsigned blocks = (unsigned)(((m->n_nodes + 3) / 4 + 7) / 8 * 8);   // a wave per node, 8 | blocks
        mpdata::unstructured::k_ustep_wave<T><<<blocks, 256, 0, st>>>(a);
    } else {
        // 16 nodes per 256-thread block (four per wave), 8 | blocks
        const int per_block = 4 * mpdata::unstructured::kNodesPerWave;
        const unsigned blocks = (unsigned)(((m->n_nodes + per_block - 1) / per_block + 7) / 8 * 8);
        mpdata::unstructured::k_ustep<T><<<blocks, 256, 0, st>>>(a);
    }
    return launch_status("unstructured step");
}

int ustep_checked(const mpdata_umesh* m, const void* psi, void* out, const void* vn, const void* w,
                  const void* rho, hipStream_t st)
{
    return m->dtype == MPDATA_F64 ? ustep<double>(m, psi, out, vn, w, rho, st)
                                  : ustep<float>(m, psi, out, vn, w, rho, st);
}

int validate_ucall(const mpdata_umesh* m, const void* psi, const void* vn, const void* w, const void* rho)
{
    if (int rc = validate_umesh(m)) return rc;
    if (int rc = check_ufield(psi, "psi", m)) return rc;
    if (m->n_edges > 0)
        if (int rc = check_ufield(vn, "vn", m)) return rc;
    if (w && !aligned(w, uelem(m))) return fail(MPDATA_EINVAL, "w is not aligned to its element size");
    return check_ufield(rho, "rho", m);
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free step (mpdata_step_noalloc): the step's
// workspace as a device array of the code object, one copy per GPU the
// library runs on, held until the process ends.  In host code `scratch`
// names a host-side stand-in: its device address on the current GPU comes
// from hipGetSymbolAddress, taken once per device and kept in
// g_scratch_addr; only that address is ever handed to a kernel.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[MPDATA_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_addr[64] = {nullptr};

// The current device's scratch address (looked up on its first use).
int scratch_address(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(MPDATA_EDEVICE, "mpdata_step_noalloc: no current device (or device index >= 64)");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MPDATA_EDEVICE, "mpdata_step_noalloc: scratch address on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return MPDATA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported entry points
// ---------------------------------------------------------------------------

extern "C" {

const char* mpdata_last_error(void) { return g_err.c_str(); }

int mpdata_ustep(const mpdata_umesh* m, const void* psi_in, void* psi_out, const void* vn, const void* w,
                 const void* rho, void* stream)
{
    if (int rc = validate_ucall(m, psi_in, vn, w, rho)) return rc;
    if (int rc = check_ufield(psi_out, "psi_out", m)) return rc;
    if (psi_in == psi_out) return fail(MPDATA_EINVAL, "psi_out must not alias psi_in");
    if (int rc = ustep_checked(m, psi_in, psi_out, vn, w, rho, (hipStream_t)stream)) return rc;
    return ok();
}

size_t mpdata_uworkspace_bytes(const mpdata_umesh* m)
{
    if (validate_umesh(m) != MPDATA_OK) return 0;
    return (((size_t)m->n_nodes * m->nz * uelem(m)) + 255) & ~(size_t)255;
}

int mpdata_urun(const mpdata_umesh* m, int32_t nsteps, void* psi, const void* vn, const void* w, const void* rho,
                void* ws, size_t ws_bytes, void* stream)
{
    if (int rc = validate_ucall(m, psi, vn, w, rho)) return rc;
    if (nsteps < 0) return fail(MPDATA_EINVAL, "nsteps=%d is negative", nsteps);
    if (!ws || !aligned(ws, 256)) return fail(MPDATA_EINVAL, "workspace is NULL or not 256-byte aligned");
    const size_t need = mpdata_uworkspace_bytes(m);
    if (ws_bytes < need) return fail(MPDATA_EINVAL, "workspace of %zu bytes is below the %zu the run needs", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    void* cur = psi;
    for (int s = 0; s < nsteps; ++s) {
        void* nxt = cur == psi ? ws : psi;
        if (int rc = ustep_checked(m, cur, nxt, vn, w, rho, st)) return rc;
        cur = nxt;
    }
    if (cur != psi) {
        hipError_t e = hipMemcpyAsync(psi, cur, (size_t)m->n_nodes * m->nz * uelem(m), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return fail(MPDATA_EDEVICE, "final copy: %s", hipGetErrorString(e));
    }
    return ok();
}

int mpdata_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (on) {   // a new record; turning timing off keeps the record for reading
        for (auto& v : g_timing.spans) {
            for (auto& pr : v) {
                g_timing.spare.push_back(pr.first);
                g_timing.spare.push_back(pr.second);
            }
            v.clear();
        }
    }
    g_timing.on = on != 0;
    return ok();
}

int mpdata_timing_read(int32_t kind, double* total_ms, int64_t* launches)
{
    if (kind < 0 || kind > 4) return fail(MPDATA_EINVAL, "timing kind %d is not an MPDATA_KERNEL_* value", kind);
    if (!total_ms || !launches) return fail(MPDATA_EINVAL, "output pointers must not be NULL");
    std::lock_guard<std::mutex> lk(g_timing.mu);
    double sum = 0.0;
    for (auto& pr : g_timing.spans[kind]) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(pr.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess) return fail(MPDATA_EDEVICE, "timing events: %s", hipGetErrorString(e));
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)g_timing.spans[kind].size();
    return ok();
}

size_t mpdata_workspace_bytes(const mpdata_problem* p, int32_t op, int32_t nsteps, int32_t checkpoint_every)
{
    if (validate(p) != MPDATA_OK) return 0;
    switch (op) {
    case MPDATA_OP_STEP: return step_bytes(p);
    case MPDATA_OP_RUN: return step_bytes(p) + field_bytes(p);
    case MPDATA_OP_MASS: return kMassBytes;
    case MPDATA_OP_ADJOINT: {
        if (nsteps < 0) { fail(MPDATA_EINVAL, "nsteps=%d is negative", nsteps); return 0; }
        int K = checkpoint_every > 0 ? checkpoint_every : (nsteps > 0 ? nsteps : 1);
        AdjLayout L = adj_layout(p, nsteps, K);
        return L.fields * L.fb;
    }
    default: fail(MPDATA_EUNSUPPORTED, "workspace query for op=%d is not supported", op); return 0;
    }
}

int mpdata_step(const mpdata_problem* p, const void* psi_in, void* psi_out, const void* cx, const void* cy,
                const void* cz, const void* g, void* ws, size_t ws_bytes, void* stream)
{
    if (int rc = validate(p)) return rc;
    if (int rc = check_ptr(psi_in, "psi_in", p)) return rc;
    if (int rc = check_ptr(psi_out, "psi_out", p)) return rc;
    if (int rc = check_ptr(cx, "cx", p)) return rc;
    if (int rc = check_ptr(cy, "cy", p)) return rc;
    if (cz && !aligned(cz, elem_size(p))) return fail(MPDATA_EINVAL, "cz is not aligned to its element size");
    if (int rc = check_ptr(g, "g", p)) return rc;
    if (psi_in == psi_out) return fail(MPDATA_EINVAL, "psi_in must not alias psi_out");
    if (!ws) return fail(MPDATA_EINVAL, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(MPDATA_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < step_bytes(p))
        return fail(MPDATA_EINVAL, "workspace of %zu bytes is below the %zu the step needs", ws_bytes, step_bytes(p));
    if (debug_on())
        if (int rc = debug_check(p->dtype, cells(p), 1, psi_in, g, ws, (hipStream_t)stream, "mpdata_step")) return rc;
    return dispatch_step(p, psi_in, psi_out, cx, cy, cz, g, ws, ws_bytes, (hipStream_t)stream);
}

int mpdata_step_noalloc(const mpdata_problem* p, const void* psi_in, void* psi_out, const void* cx, const void* cy,
                        const void* cz, const void* g, void* stream)
{
    if (int rc = validate(p)) return rc;
    if (int rc = check_ptr(psi_in, "psi_in", p)) return rc;
    if (int rc = check_ptr(psi_out, "psi_out", p)) return rc;
    if (int rc = check_ptr(cx, "cx", p)) return rc;
    if (int rc = check_ptr(cy, "cy", p)) return rc;
    if (cz && !aligned(cz, elem_size(p))) return fail(MPDATA_EINVAL, "cz is not aligned to its element size");
    if (int rc = check_ptr(g, "g", p)) return rc;
    if (psi_in == psi_out) return fail(MPDATA_EINVAL, "psi_in must not alias psi_out");
    const size_t need = step_bytes(p);
    if (need > (size_t)MPDATA_NOALLOC_SCRATCH_BYTES)
        return fail(MPDATA_EINVAL, "mpdata_step_noalloc: the step needs %zu bytes of workspace, above the %zu of "
                    "the fixed scratch (use mpdata_step with a workspace of that size)",
                    need, (size_t)MPDATA_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    if (int rc = scratch_address(&ws)) return rc;
    if (debug_on())
        if (int rc = debug_check(p->dtype, cells(p), 1, psi_in, g, ws, (hipStream_t)stream, "mpdata_step_noalloc"))
            return rc;
    return dispatch_step(p, psi_in, psi_out, cx, cy, cz, g, ws, need, (hipStream_t)stream);
}

int mpdata_run(const mpdata_problem* p, int32_t nsteps, void* psi, const void* cx, const void* cy, const void* cz,
               const void* g, void* ws, size_t ws_bytes, void* stream)
{
    if (int rc = validate(p)) return rc;
    if (nsteps < 0) return fail(MPDATA_EINVAL, "nsteps=%d is negative", nsteps);
    if (int rc = check_ptr(psi, "psi", p)) return rc;
    if (int rc = check_ptr(cx, "cx", p)) return rc;
    if (int rc = check_ptr(cy, "cy", p)) return rc;
    if (cz && !aligned(cz, elem_size(p))) return fail(MPDATA_EINVAL, "cz is not aligned to its element size");
    if (int rc = check_ptr(g, "g", p)) return rc;
    if (!ws) return fail(MPDATA_EINVAL, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(MPDATA_EINVAL, "workspace must be 256-byte aligned");
    size_t need = step_bytes(p) + field_bytes(p);
    if (ws_bytes < need)
        return fail(MPDATA_EINVAL, "workspace of %zu bytes is below the %zu the run needs", ws_bytes, need);
    if (nsteps == 0) return ok();
    hipStream_t st = (hipStream_t)stream;
    if (debug_on())
        if (int rc = debug_check(p->dtype, cells(p), 1, psi, g, ws, st, "mpdata_run")) return rc;
    void* alt = (char*)ws + step_bytes(p);
    void* cur = psi;
    for (int s = 0; s < nsteps; ++s) {
        void* nxt = (cur == psi) ? alt : psi;
        if (int rc = dispatch_step(p, cur, nxt, cx, cy, cz, g, ws, step_bytes(p), st)) return rc;
        cur = nxt;
    }
    if (cur != psi) {
        hipError_t e = hipMemcpyAsync(psi, cur, (size_t)cells(p) * elem_size(p), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return fail(MPDATA_EDEVICE, "final copy: %s", hipGetErrorString(e));
    }
    return ok();
}

int mpdata_adjoint(const mpdata_problem* p, int32_t nsteps, int32_t checkpoint_every, const void* psi0,
                   const void* cx, const void* cy, const void* cz, const void* g, const void* dJ_dpsiT,
                   void* dJ_dpsi0, void* dJ_dcx, void* dJ_dcy, void* dJ_dcz, void* psiT_out, void* ws,
                   size_t ws_bytes, void* stream)
{
    if (int rc = validate(p)) return rc;
    if (p->dtype != MPDATA_F64) return fail(MPDATA_EUNSUPPORTED, "the adjoint is implemented in FP64 only");
    if (nsteps < 0) return fail(MPDATA_EINVAL, "nsteps=%d is negative", nsteps);
    if (checkpoint_every < 0) return fail(MPDATA_EINVAL, "checkpoint_every=%d is negative", checkpoint_every);
    const void* req[] = {psi0, cx, cy, g, dJ_dpsiT, dJ_dpsi0, dJ_dcx, dJ_dcy};
    const char* names[] = {"psi0", "cx", "cy", "g", "dJ_dpsiT", "dJ_dpsi0", "dJ_dcx", "dJ_dcy"};
    for (int e = 0; e < 8; ++e)
        if (int rc = check_ptr(req[e], names[e], p)) return rc;
    if (cz && !aligned(cz, 8)) return fail(MPDATA_EINVAL, "cz is not aligned to its element size");
    if (dJ_dcz && !aligned(dJ_dcz, 8)) return fail(MPDATA_EINVAL, "dJ_dcz is not aligned to its element size");
    if (psiT_out && !aligned(psiT_out, 8)) return fail(MPDATA_EINVAL, "psiT_out is not aligned");
    {
        // no output may alias an input or another output: the sweep writes its
        // outputs while it still reads the inputs (the seed is copied, the
        // wind gradients are cleared, before the segments are recomputed)
        const void* in[] = {psi0, cx, cy, cz, g, dJ_dpsiT};
        const char* in_names[] = {"psi0", "cx", "cy", "cz", "g", "dJ_dpsiT"};
        const void* out[] = {dJ_dpsi0, dJ_dcx, dJ_dcy, dJ_dcz, psiT_out};
        const char* out_names[] = {"dJ_dpsi0", "dJ_dcx", "dJ_dcy", "dJ_dcz", "psiT_out"};
        for (int o = 0; o < 5; ++o) {
            if (!out[o]) continue;
            for (int i = 0; i < 6; ++i)
                if (out[o] == in[i])
                    return fail(MPDATA_EINVAL, "%s must not alias the input %s", out_names[o], in_names[i]);
            for (int o2 = 0; o2 < o; ++o2)
                if (out[o] == out[o2])
                    return fail(MPDATA_EINVAL, "%s must not alias the output %s", out_names[o], out_names[o2]);
            if (out[o] == ws) return fail(MPDATA_EINVAL, "%s must not alias the workspace", out_names[o]);
        }
    }
    if (!ws || !aligned(ws, 256)) return fail(MPDATA_EINVAL, "workspace is NULL or not 256-byte aligned");
    const int K = checkpoint_every > 0 ? checkpoint_every : (nsteps > 0 ? nsteps : 1);
    const AdjLayout L = adj_layout(p, nsteps, K);
    if (ws_bytes < L.fields * L.fb)
        return fail(MPDATA_EINVAL, "workspace of %zu bytes is below the %zu the adjoint needs", ws_bytes,
                    L.fields * L.fb);
    if (debug_on())
        if (int rc = debug_check(p->dtype, cells(p), 1, psi0, g, ws, (hipStream_t)stream, "mpdata_adjoint"))
            return rc;
    return adjoint_run(p, nsteps, K, (const double*)psi0, (const double*)cx, (const double*)cy, (const double*)cz,
                       (const double*)g, (const double*)dJ_dpsiT, (double*)dJ_dpsi0, (double*)dJ_dcx,
                       (double*)dJ_dcy, (double*)dJ_dcz, (double*)psiT_out, ws, (hipStream_t)stream);
}

size_t mpdata_batch_workspace_bytes(const mpdata_problem* common, int32_t nitems, const mpdata_batch_item* items)
{
    if (!common) { fail(MPDATA_EINVAL, "problem pointer is NULL"); return 0; }
    mpdata_problem c = *common;
    c.nx = c.ny = c.nz = 1;
    if (validate(&c) != MPDATA_OK) return 0;
    if (validate_items(&c, nitems, items) != MPDATA_OK) return 0;
    return batch::layout(&c, nitems, items).total;
}

int mpdata_run_batched(const mpdata_problem* common, int32_t nitems, const mpdata_batch_item* items,
                       int32_t nsteps, int32_t flags, void* ws, size_t ws_bytes, void* stream)
{
    if (!common) return fail(MPDATA_EINVAL, "problem pointer is NULL");
    mpdata_problem c = *common;
    c.nx = c.ny = c.nz = 1;   // sizes come from the items
    if (int rc = validate(&c)) return rc;
    if (int rc = validate_items(&c, nitems, items)) return rc;
    if (nsteps < 0) return fail(MPDATA_EINVAL, "nsteps=%d is negative", nsteps);
    if (flags & ~(MPDATA_BATCH_GRAPH | MPDATA_BATCH_TUNE)) return fail(MPDATA_EINVAL, "unknown flags 0x%x", flags);
    if (c.iters > 9) return fail(MPDATA_EUNSUPPORTED, "batched runs support up to 9 passes");
    if (!ws || !aligned(ws, 256)) return fail(MPDATA_EINVAL, "workspace is NULL or not 256-byte aligned");
    const batch::Layout L = batch::layout(&c, nitems, items);
    if (ws_bytes < L.total)
        return fail(MPDATA_EINVAL, "workspace of %zu bytes is below the %zu the batch needs", ws_bytes, L.total);
    if (nsteps == 0) return ok();
    if (debug_on())
        for (int i = 0; i < nitems; ++i) {
            char who[64];
            snprintf(who, sizeof who, "mpdata_run_batched item %d", i);
            const long long n = (long long)items[i].nx * items[i].ny * items[i].nz;
            if (int rc = debug_check(c.dtype, n, items[i].ntracers, items[i].psi, items[i].g, ws, (hipStream_t)stream,
                                     who))
                return rc;
        }
    if (c.dtype == MPDATA_F64) return run_batched<double>(&c, nitems, items, nsteps, flags, ws, (hipStream_t)stream);
    return run_batched<float>(&c, nitems, items, nsteps, flags, ws, (hipStream_t)stream);
}

int mpdata_mass(const mpdata_problem* p, const void* psi, const void* g, double* host_out, void* ws,
                size_t ws_bytes, void* stream)
{
    if (int rc = validate(p)) return rc;
    if (int rc = check_ptr(psi, "psi", p)) return rc;
    if (int rc = check_ptr(g, "g", p)) return rc;
    if (!host_out) return fail(MPDATA_EINVAL, "host_out is NULL");
    if (!ws || !aligned(ws, 8)) return fail(MPDATA_EINVAL, "workspace is NULL or misaligned");
    if (ws_bytes < kMassBytes)
        return fail(MPDATA_EINVAL, "workspace of %zu bytes is below the %zu the mass needs", ws_bytes, kMassBytes);
    hipStream_t st = (hipStream_t)stream;
    double* part = (double*)ws;
    if (p->dtype == MPDATA_F64)
        k_mass_partial<double><<<kMassBlocks, kMassThreads, 0, st>>>(cells(p), (const double*)psi,
                                                                      (const double*)g, part);
    else
        k_mass_partial<float><<<kMassBlocks, kMassThreads, 0, st>>>(cells(p), (const float*)psi,
                                                                     (const float*)g, part);
    if (int rc = launch_status("mass partial sums")) return rc;
    k_mass_final<<<1, kMassThreads, 0, st>>>(kMassBlocks, part);
    if (int rc = launch_status("mass final sum")) return rc;
    hipError_t e = hipMemcpyAsync(host_out, part + 2 * kMassBlocks, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(MPDATA_EDEVICE, "mass read-back: %s", hipGetErrorString(e));
    return ok();
}

}  // extern "C"
