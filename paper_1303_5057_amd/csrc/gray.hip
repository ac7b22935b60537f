// gray.hip -- HIP kernels and C ABI (include/gray.h) of the MI355X Kerr
// photon-geodesic integrator.
//
// Scheme (Chan, Psaltis & Ozel 2013, Sec. 2): classical RK4 on the 8-component
// second-order geodesic equation, the step-size rule of eq. (2), the horizon
// stop, the theta remap of eq. (3) and the null-condition monitor of eq. (4)
// with a forward-Euler re-integration at h / 9.
//
// GPU design: one photon per lane of a 64-wide wavefront, state in VGPRs for
// the whole trajectory, structure-of-arrays state in HBM read once and written
// once per photon. The integrate kernel is persistent: a wave holds 64 photons,
// and whenever lanes have finished it hands them the next photon ids of a
// chunk taken from one global counter, so lanes stay busy while step counts
// differ per photon. The ids come from the caller's work list or, in dense
// mode, from a launch order that starts the photons expected to take the most
// steps first (k_order_key).
#include "../../include/gray.h"
#include "kerr.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <utility>
#include <vector>
#include <cstdio>
#include <cstring>
#include <mutex>

namespace gray {

static_assert(kPoleMonitor == GRAY_POLE_MONITOR && kPoleEulerCrossing == GRAY_POLE_EULER_CROSSING &&
                  kPoleNone == GRAY_POLE_NONE,
              "pole treatments match gray_pole_mode");

// ------------------------------------------------------------------ errors
static thread_local char g_last_error[512] = "no device error";

static int device_error(const char *what, hipError_t e)
{
    snprintf(g_last_error, sizeof g_last_error, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return GRAY_EDEVICE;
}

static int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GRAY_OK : device_error(what, e);
}

// ------------------------------------------------------------ constants
constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kCamChunk = 16;          // cameras per by-value kernel argument
constexpr unsigned kQueueChunk = 64;   // photons per refill round (one per lane)
constexpr unsigned kMaxGrab = 8;       // refill rounds per queue grab, at most
constexpr unsigned kSpan = 512;        // work-list ids reserved per append grab
constexpr int64_t kMaxListWaves = 2048; // waves of a work-list launch, at most
static_assert(kMaxListWaves * kSpan <= GRAY_WORKLIST_SLACK, "list slack covers every wave's last span");
constexpr size_t kWsHeader = 512;      // WsHeader, padded
constexpr int kOrderBins = 32;         // scheduling-key buckets
constexpr unsigned kOrderBlocks = 2048; // blocks of the ordering passes, at most
static_assert(GRAY_MAX_PHOTONS + (int64_t)(kQueueChunk * kMaxGrab + kSpan) < ((int64_t)1 << 31),
              "ids, queue positions and their overshoot fit in 32 bits");

// Start of the workspace: queue counter and the ordering pass's counts.
struct WsHeader {
    unsigned long long queue;       // positions handed out: from the head (low
                                    // 32 bits) and from the tail (high 32 bits)
    unsigned count;                 // photons in the launch order
    unsigned pad[29];
    unsigned hist[kOrderBins];      // running photons per key bucket
    unsigned cursor[kOrderBins];    // positions handed out per bucket
};
static_assert(sizeof(WsHeader) <= kWsHeader, "header fits its reserved space");

// Per-camera constants the integrator needs, kept in the workspace.
struct DevCam {
    double a, a2, rbh, rcap, disk_rmin, disk_rmax, eps3;
    int32_t call_steps;   // per-camera step budget of a call (0: the call's)
    int32_t pad;
};
static_assert(sizeof(DevCam) == 64, "DevCam is one 64-byte record");

// Camera geometry passed by value to the init and classify kernels.
struct CamArg {
    double a, r_obs, incl, alo, ahi, blo, bhi, eps3;
    int64_t first;
    int32_t nx, ny, index, kind, metric, pad;
};
struct CamChunk {
    CamArg c[kCamChunk];
    int32_t count;
    int32_t sparse;   // slot mode: photons in [lo, hi) may belong to no camera here
    int64_t lo, hi;   // photon range [lo, hi) covered by these cameras
};
struct SetupChunk {
    DevCam c[kCamChunk];
    int32_t base, count;
};

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ unsigned lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Camera of photon i within a chunk, or -1 (slot mode only) when none covers it.
__device__ __forceinline__ int find_camera(const CamChunk &ch, int64_t i)
{
    if (ch.sparse) {
        for (int j = 0; j < ch.count; ++j)
            if (i >= ch.c[j].first && i < ch.c[j].first + (int64_t)ch.c[j].nx * ch.c[j].ny) return j;
        return -1;
    }
    int k = 0;
    for (int j = 1; j < ch.count; ++j)
        if (i >= ch.c[j].first) k = j;
    return k;
}

// Image-plane coordinates of photon i of camera c (see gray_camera).
__device__ __forceinline__ void pixel_of(const CamArg &c, int64_t i, double &alpha, double &beta)
{
    const int64_t local = i - c.first;
    const int32_t iy = (int32_t)(local / c.nx);
    const int32_t ix = (int32_t)(local - (int64_t)iy * c.nx);
    const double u = c.alo + (c.ahi - c.alo) * ((ix + 0.5) / c.nx);
    if (c.kind == GRAY_CAMERA_POLAR) {
        const double th = c.ny > 1 ? c.blo + (c.bhi - c.blo) * ((double)iy / (c.ny - 1)) : c.blo;
        double s, co;
        sincos(th, &s, &co);
        alpha = u * co;
        beta = u * s;
    } else {
        alpha = u;
        beta = c.blo + (c.bhi - c.blo) * ((iy + 0.5) / c.ny);
    }
}

// ------------------------------------------------------- camera initialisation
struct InitArgs {
    void *x, *lo;
    int32_t *status, *steps, *cam, *counters;
    double *mark, *disk;
    int32_t *work;          // work-list mode: append initialised ids here
    unsigned *work_count;
    unsigned *cam_done;     // zeroed for the cameras of the chunk
    int64_t stride;
    int32_t precision, pad;
    CamChunk ch;
};

__global__ __launch_bounds__(kBlock) void k_camera_init(InitArgs A)
{
    if (A.cam_done && blockIdx.x == 0 && threadIdx.x < (unsigned)A.ch.count)
        A.cam_done[A.ch.c[threadIdx.x].index] = 0u;
    const int64_t i = A.ch.lo + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.ch.hi) return;
    const int kc = find_camera(A.ch, i);
    if (kc < 0) return;
    const CamArg &c = A.ch.c[kc];
    double alpha, beta;
    pixel_of(c, i, alpha, beta);
    State<double> x;
    camera_state(c.a, c.r_obs, c.incl, alpha, beta, x, c.eps3, c.metric == GRAY_METRIC_DEFORMED);
    const int64_t S = A.stride;
    if (A.precision == GRAY_FP64) {
        double *X = (double *)A.x;
        for (int k = 0; k < 8; ++k) X[k * S + i] = get(x, k);
    } else {
        float *H = (float *)A.x, *L = (float *)A.lo;
        for (int k = 0; k < 8; ++k) {
            const double v = get(x, k);
            const float hi = (float)v;
            H[k * S + i] = hi;
            L[k * S + i] = (float)(v - (double)hi);
        }
    }
    A.status[i] = GRAY_RUNNING;
    A.steps[i] = 0;
    A.cam[i] = c.index;
    if (A.counters)
        for (int k = 0; k < 3; ++k) A.counters[k * S + i] = 0;
    if (A.mark) A.mark[1 * S + i] = 0.0;
    if (A.disk)
        for (int k = 0; k < 3; ++k) A.disk[k * S + i] = 0.0;
    if (A.work) {
        const uint64_t m = ballot(true);
        const unsigned lane = threadIdx.x & (kWave - 1);
        unsigned base = 0;
        if (lane == (unsigned)(__ffsll((long long)m) - 1)) base = atomicAdd(A.work_count, (unsigned)__popcll(m));
        base = __builtin_amdgcn_readfirstlane(base);
        A.work[base + lane_rank(m)] = (int32_t)i;
    }
}

// ------------------------------------------------------------ workspace setup
__global__ void k_setup(DevCam *table, WsHeader *hdr, unsigned *work_out_count, SetupChunk ch)
{
    const int j = threadIdx.x;
    if (j < ch.count) table[ch.base + j] = ch.c[j];
    if (ch.base == 0) {
        if (j < kOrderBins) {
            hdr->hist[j] = 0u;
            hdr->cursor[j] = 0u;
        }
        if (j == 0) {
            hdr->queue = 0u;
            hdr->count = 0u;
            if (work_out_count) *work_out_count = 0u;
        }
    }
}

// ------------------------------------------------------------ launch order
// Step counts differ by an order of magnitude between photons, and a launch
// lasts at least as long as its longest photon takes after it starts. The
// dense-mode launch therefore hands out photons in increasing order of a key
// that is small for the photons expected to take the most steps:
//  * those that circle the hole near a spherical photon orbit. With
//    lam = L / E and eta = Q / E^2 the radial potential is
//      R(r) = r^4 + (a^2 - eta - lam^2) r^2 + 2 (eta + (lam - a)^2) r - a^2 eta,
//    and a double root of R outside the horizon is such an orbit; the first
//    factor of the key is |R| / r^4 at R's outer local minimum (not inside the
//    horizon), or 1 when R has no local minimum at r > 0;
//  * those with small |L_z|, which pass near the polar axis, where the
//    step-size rule of eq. (2) shrinks the step (k^phi grows like
//    L / sin^2 theta) and the null monitor of eq. (4) trips; the second factor
//    is |lam| / (|lam| + 1).
// The order changes which lane advances a photon and when, never the
// photon's result.
__device__ double order_key(double a, double rbh, const State<double> &x)
{
    double E, L, Q;
    conserved(a, x, E, L, Q);
    const double lam = L / E, eta = Q / (E * E);
    const double pole = fabs(lam) / (fabs(lam) + 1.0);
    const double A2 = a * a - eta - lam * lam;
    const double B1 = 2.0 * (eta + (lam - a) * (lam - a));
    const double C0 = -a * a * eta;
    if (!(A2 < 0.0)) return pole;
    // R'(r) = 4 r^3 + 2 A2 r + B1 is convex right of R's inflection point
    // ri; a local minimum of R exists there iff R'(ri) < 0, and Newton's
    // method from r0 = sqrt(-A2 / 2) > ri converges to it without leaving
    // the convex part.
    const double ri = sqrt(-A2 / 6.0);
    if (!((4.0 * ri * ri + 2.0 * A2) * ri + B1 < 0.0)) return pole;
    double r = sqrt(-A2 / 2.0);
    for (int k = 0; k < 8; ++k) r -= ((4.0 * r * r + 2.0 * A2) * r + B1) / (12.0 * r * r + 2.0 * A2);
    r = fmax(r, rbh);
    const double r2 = r * r;
    return pole * fabs(((r2 + A2) * r2 + B1 * r + C0) / (r2 * r2));
}

// Bucket of a key: its binary exponent, so keys 2^-24 .. 2^7 spread over
// kOrderBins buckets; non-finite keys go last.
__device__ __forceinline__ unsigned order_bucket(double key)
{
    if (!(key < 128.0)) return kOrderBins - 1;
    if (key < 0x1p-24) return 0;
    int e;
    frexp(key, &e);
    return (unsigned)min(max(e + 24, 0), kOrderBins - 1);
}

struct OrderArgs {
    const void *x, *lo;
    const int32_t *status, *cam;
    const DevCam *cams;
    uint8_t *bucket;        // per photon: key bucket, or 0xff when not running
    unsigned *block_hist;   // per ordering block and bucket
    int32_t *perm;          // launch order of the running photons
    WsHeader *hdr;
    int64_t n, stride, per_block;
    int32_t precision, pad;
};

// Pass 1: bucket of every running photon, per-block and global histograms.
__global__ __launch_bounds__(kBlock) void k_order_key(OrderArgs A)
{
    __shared__ unsigned h[kOrderBins];
    if (threadIdx.x < kOrderBins) h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * A.per_block;
    const int64_t i1 = i0 + A.per_block < A.n ? i0 + A.per_block : A.n;
    const int64_t S = A.stride;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
        unsigned b = 0xffu;
        if (A.status[i] == GRAY_RUNNING) {
            State<double> x;
            double v[8];
            if (A.precision == GRAY_FP64) {
                const double *X = (const double *)A.x;
                for (int k = 0; k < 8; ++k) v[k] = X[k * S + i];
            } else {
                const float *H = (const float *)A.x, *L = (const float *)A.lo;
                for (int k = 0; k < 8; ++k) v[k] = (double)H[k * S + i] + (double)L[k * S + i];
            }
            x.t = v[0]; x.r = v[1]; x.th = v[2]; x.ph = v[3];
            x.kt = v[4]; x.kr = v[5]; x.kth = v[6]; x.kph = v[7];
            const DevCam cm = A.cams[A.cam[i]];
            b = order_bucket(order_key(cm.a, cm.rbh, x));
            atomicAdd(&h[b], 1u);
        }
        A.bucket[i] = (uint8_t)b;
    }
    __syncthreads();
    if (threadIdx.x < kOrderBins) {
        const unsigned c = h[threadIdx.x];
        A.block_hist[(int64_t)blockIdx.x * kOrderBins + threadIdx.x] = c;
        if (c) {
            atomicAdd(&A.hdr->hist[threadIdx.x], c);
            atomicAdd(&A.hdr->count, c);
        }
    }
}

// Pass 2: each block reserves, per bucket, room for its photons after the
// buckets before it, then writes their ids. The lanes of a wave that share
// a bucket take consecutive positions in lane (= id) order, so the order
// holds runs of nearby ids and the integrator's state loads stay mostly
// coalesced; the order of the runs inside a bucket is arbitrary.
__global__ __launch_bounds__(kBlock) void k_order_scatter(OrderArgs A)
{
    __shared__ unsigned base[kOrderBins], run[kOrderBins];
    const unsigned j = threadIdx.x;
    if (j < kOrderBins) {
        unsigned start = 0;
        for (unsigned k = 0; k < j; ++k) start += A.hdr->hist[k];
        const unsigned c = A.block_hist[(int64_t)blockIdx.x * kOrderBins + j];
        base[j] = c ? start + atomicAdd(&A.hdr->cursor[j], c) : 0u;
        run[j] = 0u;
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * A.per_block;
    const int64_t i1 = i0 + A.per_block < A.n ? i0 + A.per_block : A.n;
    const unsigned lane = threadIdx.x & (kWave - 1);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const unsigned b = A.bucket[i];
        bool todo = b < (unsigned)kOrderBins;
        for (;;) {
            const uint64_t m = ballot(todo);
            if (m == 0ull) break;
            const int lead = __ffsll((long long)m) - 1;
            const unsigned bl = (unsigned)__shfl((int)b, lead, kWave);
            const bool mine = todo && b == bl;
            const uint64_t same = ballot(mine);
            unsigned at = 0;
            if ((int)lane == lead) at = atomicAdd(&run[bl], (unsigned)__popcll(same));
            at = (unsigned)__shfl((int)at, lead, kWave);
            if (mine) {
                A.perm[base[bl] + at + lane_rank(same)] = (int32_t)i;
                todo = false;
            }
        }
    }
}


// ------------------------------------------------------- persistent integrator
struct IntArgs {
    void *x, *lo;
    int32_t *status, *steps;
    const int32_t *cam;
    int32_t *counters;
    double *mark, *disk;
    const DevCam *cams;
    unsigned long long *queue;  // WsHeader::queue
    const int32_t *work_in;     // ids to advance (the caller's work list or the launch order), count at *work_in_count
    int32_t *work_out;          // ids still running at the end, count at *work_out_count
    const unsigned *work_in_count;
    unsigned *work_out_count;
    unsigned *cam_done;         // per-camera count of photons that stopped
    unsigned long long *wave_iters; // += loop iterations with a busy lane
    int64_t n, stride;
    double step_frac, xi_eps, euler_inv, r_escape;
    double fp64_horizon, fp64_pole, fp64_turn;
    int32_t max_steps, call_steps;
    uint32_t flags;
    int32_t refill;
    int32_t two_ended;          // odd wave slots take ids from the end of the queue
    int32_t helper;             // FP32C: the FP64 wave may run float photons
    int32_t pad;
    const unsigned *stop;       // host-set stop request, or null
};

// Argument block fields of the running k_integrate, read again where they
// are used. The persistent loop needs most of its pointers only when a
// photon starts or stops; held in scalar registers across the loop, they and
// the per-component addresses the compiler derives from them would crowd
// out the stepping code's own scalar values (its sin/cos coefficients) and
// spill. A scalar load from the kernel-argument segment inside an asm
// statement can be neither hoisted nor combined. Valid only in kernels
// whose sole argument is an IntArgs.
template <class T, size_t OFF>
__device__ __forceinline__ T int_arg()
{
    static_assert(sizeof(T) == 8, "64-bit fields only");
    const auto kp = __builtin_amdgcn_kernarg_segment_ptr();
    T v;
    asm volatile("s_load_dwordx2 %0, %1, %2\n\ts_waitcnt lgkmcnt(0)" : "=s"(v) : "s"(kp), "i"(OFF));
    return v;
}
#define GRAY_ARG(f) int_arg<decltype(IntArgs::f), offsetof(IntArgs, f)>()

// The pointer fields of IntArgs (its first 128 bytes), read back with one
// or two scalar loads and a single wait: the eight per-photon arrays, and
// the camera table and queue pointers.
struct ArgPointers {
    void *x, *lo;
    int32_t *status, *steps;
    const int32_t *cam;
    int32_t *counters;
    double *mark, *disk;
    const DevCam *cams;
    unsigned long long *queue;
    const int32_t *work_in;
    int32_t *work_out;
    const unsigned *work_in_count;
    unsigned *work_out_count;
    unsigned *cam_done;
    unsigned long long *wave_iters;
};
static_assert(sizeof(ArgPointers) == 128 && offsetof(IntArgs, x) == 0 && offsetof(IntArgs, lo) == 8 &&
                  offsetof(IntArgs, status) == 16 && offsetof(IntArgs, steps) == 24 &&
                  offsetof(IntArgs, cam) == 32 && offsetof(IntArgs, counters) == 40 &&
                  offsetof(IntArgs, mark) == 48 && offsetof(IntArgs, disk) == 56 &&
                  offsetof(IntArgs, cams) == 64 && offsetof(IntArgs, queue) == 72 &&
                  offsetof(IntArgs, work_in) == 80 && offsetof(IntArgs, work_out) == 88 &&
                  offsetof(IntArgs, work_in_count) == 96 && offsetof(IntArgs, work_out_count) == 104 &&
                  offsetof(IntArgs, cam_done) == 112 && offsetof(IntArgs, wave_iters) == 120,
              "ArgPointers mirrors the first 128 bytes of IntArgs");

// N = 1: the per-photon arrays only (the rest left null); N = 2: all.
template <int N>
__device__ __forceinline__ ArgPointers arg_pointers()
{
    typedef unsigned u32x16 __attribute__((ext_vector_type(16)));
    const auto kp = __builtin_amdgcn_kernarg_segment_ptr();
    u32x16 v0, v1 = {};
    if constexpr (N == 1)
        asm volatile("s_load_dwordx16 %0, %1, 0\n\ts_waitcnt lgkmcnt(0)" : "=s"(v0) : "s"(kp));
    else
        asm volatile("s_load_dwordx16 %0, %2, 0\n\ts_load_dwordx16 %1, %2, 64\n\ts_waitcnt lgkmcnt(0)"
                     : "=&s"(v0), "=&s"(v1)
                     : "s"(kp));
    ArgPointers P;
    uint64_t *w = (uint64_t *)&P;
    for (int k = 0; k < 8; ++k) w[k] = (uint64_t)v0[2 * k] | ((uint64_t)v0[2 * k + 1] << 32);
    for (int k = 0; k < 8; ++k) w[8 + k] = (uint64_t)v1[2 * k] | ((uint64_t)v1[2 * k + 1] << 32);
    return P;
}

template <class T>
using global_ptr = __attribute__((address_space(1))) T *;

// The same pointer as a global-memory one (accesses through a pointer read
// back by int_arg would otherwise be generic, flat ones).
template <class T>
__device__ __forceinline__ global_ptr<T> glob(T *p) { return (global_ptr<T>)p; }

// Element id of a component-major array of stride S, visited one component
// after the other. The address advances in vector registers through an
// empty asm statement, so the compiler cannot replace the walk by one
// scalar base address per component.
template <class T>
struct Column {
    global_ptr<T> p;
    int64_t S;
    __device__ __forceinline__ Column(T *base, int64_t stride, int64_t id) : p((global_ptr<T>)base + id), S(stride) {}
    __device__ __forceinline__ T get() const { return *p; }
    __device__ __forceinline__ void put(T v) const { *p = v; }
    __device__ __forceinline__ void next()
    {
        p += S;
        asm volatile("" : "+v"(p));
    }
};

// Per-lane photon of the persistent loop. In FP64 the state is x; in FP32C
// it is hi + lo (floats) and x is not kept between steps.
template <int P>
struct Lane;

template <>
struct Lane<GRAY_FP64> {
    State<double> x;
    double s, c;
    __device__ __forceinline__ void load(const void *xp, const void *, int64_t S, int64_t id)
    {
        Column<const double> X((const double *)xp, S, id);
        double v[8];
        for (int k = 0; k < 8; ++k) {
            v[k] = X.get();
            if (k < 7) X.next();
        }
        x.t = v[0]; x.r = v[1]; x.th = v[2]; x.ph = v[3];
        x.kt = v[4]; x.kr = v[5]; x.kth = v[6]; x.kph = v[7];
        sin_cos(x.th, s, c);
    }
    __device__ __forceinline__ void store(void *xp, void *, int64_t S, int64_t id) const
    {
        const double v[8] = {x.t, x.r, x.th, x.ph, x.kt, x.kr, x.kth, x.kph};
        Column<double> X((double *)xp, S, id);
        for (int k = 0; k < 8; ++k) {
            X.put(v[k]);
            if (k < 7) X.next();
        }
    }
    __device__ __forceinline__ State<double> value() const { return x; }
};

template <>
struct Lane<GRAY_FP32C> {
    State<float> hi, lo;
    float s, c;   // sin and cos of hi.th + lo.th
    __device__ __forceinline__ void load(const void *hp, const void *lp, int64_t S, int64_t id)
    {
        Column<const float> H((const float *)hp, S, id), L((const float *)lp, S, id);
        float h[8], l[8];
        for (int k = 0; k < 8; ++k) {
            h[k] = H.get();
            l[k] = L.get();
            if (k < 7) {
                H.next();
                L.next();
            }
        }
        hi.t = h[0]; hi.r = h[1]; hi.th = h[2]; hi.ph = h[3]; hi.kt = h[4]; hi.kr = h[5]; hi.kth = h[6]; hi.kph = h[7];
        lo.t = l[0]; lo.r = l[1]; lo.th = l[2]; lo.ph = l[3]; lo.kt = l[4]; lo.kr = l[5]; lo.kth = l[6]; lo.kph = l[7];
        sincos_full_lo(hi.th, lo.th, s, c);
    }
    __device__ __forceinline__ void store(void *hp, void *lp, int64_t S, int64_t id) const
    {
        const float h[8] = {hi.t, hi.r, hi.th, hi.ph, hi.kt, hi.kr, hi.kth, hi.kph};
        const float l[8] = {lo.t, lo.r, lo.th, lo.ph, lo.kt, lo.kr, lo.kth, lo.kph};
        Column<float> H((float *)hp, S, id), L((float *)lp, S, id);
        for (int k = 0; k < 8; ++k) {
            H.put(h[k]);
            L.put(l[k]);
            if (k < 7) {
                H.next();
                L.next();
            }
        }
    }
    __device__ __forceinline__ State<double> value() const
    {
        State<double> x;
        x.t = (double)hi.t + (double)lo.t; x.r = (double)hi.r + (double)lo.r;
        x.th = (double)hi.th + (double)lo.th; x.ph = (double)hi.ph + (double)lo.ph;
        x.kt = (double)hi.kt + (double)lo.kt; x.kr = (double)hi.kr + (double)lo.kr;
        x.kth = (double)hi.kth + (double)lo.kth; x.kph = (double)hi.kph + (double)lo.kph;
        return x;
    }
    // hi + lo nearest x (to about 48 bits), without sin/cos
    __device__ __forceinline__ void split(const State<double> &x)
    {
#define GRAY_SPLIT(cmp) hi.cmp = (float)x.cmp; lo.cmp = (float)(x.cmp - (double)hi.cmp)
        GRAY_SPLIT(t); GRAY_SPLIT(r); GRAY_SPLIT(th); GRAY_SPLIT(ph);
        GRAY_SPLIT(kt); GRAY_SPLIT(kr); GRAY_SPLIT(kth); GRAY_SPLIT(kph);
#undef GRAY_SPLIT
    }
    __device__ __forceinline__ void set(const State<double> &x)
    {
        split(x);
        sincos_full_lo(hi.th, lo.th, s, c);
    }
};

__device__ __forceinline__ bool finite_state(const State<double> &x)
{
    return isfinite(x.t) && isfinite(x.r) && isfinite(x.th) && isfinite(x.ph) && isfinite(x.kt) &&
           isfinite(x.kr) && isfinite(x.kth) && isfinite(x.kph);
}

// Stop bookkeeping of the persistent loops, once per iteration (a
// wave-uniform call): work-list output of the photons still running, written
// into a private span of kSpan reserved slots per wave (when it fills up the
// rest continues in a fresh span, so the only unused slots are the tail of
// each wave's last span, marked -1 at exit), and the per-camera completion
// counts (one atomic per wave when the photons that finished share a camera).
struct StopBook {
    unsigned span_next = 0, span_end = 0;
    __device__ __forceinline__ void account(bool stop_now, bool keep, int64_t id, unsigned lane, bool list_out,
                                            bool count_done)
    {
        if (list_out) {
            const uint64_t m = ballot(keep);
            const unsigned cnt = (unsigned)__popcll(m);
            if (cnt) {
                const unsigned room = span_end - span_next;
                unsigned fresh = 0;
                if (cnt > room) {
                    if (lane == 0) fresh = atomicAdd(GRAY_ARG(work_out_count), kSpan);
                    fresh = __builtin_amdgcn_readfirstlane(fresh);
                }
                const unsigned r = lane_rank(m);
                if (keep) glob(GRAY_ARG(work_out))[r < room ? span_next + r : fresh + (r - room)] = (int32_t)id;
                if (cnt > room) {
                    span_next = fresh + (cnt - room);
                    span_end = fresh + kSpan;
                } else {
                    span_next += cnt;
                }
            }
        }
        if (count_done) {
            const bool fin = stop_now && !keep;
            const uint64_t mf = ballot(fin);
            if (mf) {
                const int32_t c = fin ? glob(GRAY_ARG(cam))[id] : -1;
                const unsigned lead = (unsigned)(__ffsll((long long)mf) - 1);
                const int32_t cl = __shfl(c, (int)lead, kWave);
                if (ballot(fin && c != cl) == 0ull) {
                    if (lane == lead) atomicAdd(GRAY_ARG(cam_done) + cl, (unsigned)__popcll(mf));
                } else if (fin) {
                    atomicAdd(GRAY_ARG(cam_done) + c, 1u);
                }
            }
        }
    }
    __device__ __forceinline__ void finish(unsigned lane, bool list_out, unsigned long long iters)
    {
        if (list_out) {
            global_ptr<int32_t> wo = glob(GRAY_ARG(work_out));
            for (unsigned j = span_next + lane; j < span_end; j += kWave) wo[j] = -1;
        }
        if (unsigned long long *wi = GRAY_ARG(wave_iters))
            if (lane == 0 && iters) atomicAdd(wi, iters);
    }
};

// One grab from the two-ended queue of ids: one atomic on the (head, tail)
// pair. With h ids taken from the head and t from the tail before this grab,
// the free positions are [h, nq - t): a head grab takes the first `grab` of
// them, a tail grab the last; every position is handed out exactly once, and
// the grab that brings h + t to nq or beyond (and every later one) finds the
// queue empty. The wave's chunk becomes [chunk_next, chunk_end). Wave-uniform.
__device__ __forceinline__ void queue_grab(unsigned lane, bool from_tail, unsigned grab, int64_t nq,
                                           bool &exhausted, unsigned &chunk_next, unsigned &chunk_end)
{
    unsigned long long old = 0;
    if (lane == 0)
        old = atomicAdd(GRAY_ARG(queue), from_tail ? (unsigned long long)grab << 32 : (unsigned long long)grab);
    const int64_t h = __builtin_amdgcn_readfirstlane((unsigned)old);
    const int64_t t = __builtin_amdgcn_readfirstlane((unsigned)(old >> 32));
    const int64_t end = nq - t;
    if (h + t + grab >= nq) exhausted = true;
    int64_t lo = h, hi = h;
    if (end > h) {
        if (from_tail) {
            hi = end;
            lo = end - grab > h ? end - grab : h;
        } else {
            hi = h + grab < end ? h + grab : end;
        }
    }
    chunk_next = (unsigned)lo;
    chunk_end = (unsigned)hi;
}

// The host-set stop request (gray_state::stop, non-null), read past the
// caches. Wave-uniform.
__device__ __forceinline__ bool stop_requested()
{
    const unsigned v = __hip_atomic_load((unsigned *)GRAY_ARG(stop), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return __builtin_amdgcn_readfirstlane(v) != 0u;
}

// Persistent integrator (FP64). Each wave keeps 64 photons in registers;
// whenever at least A.refill lanes are idle it hands them the next photons of
// the wave's current chunk of the queue, taking a new chunk from the global
// counter when the old one is used up. A wave exits once the counter is past
// the queue length and all its lanes are idle; every photon ends within
// max_steps (or call_steps) steps, so every wave exits. PM is the treatment of
// the polar axis (the production monitor unless a caller asks for one of the
// paper's earlier treatments), a template parameter so that the production
// kernel carries no code for the others; MET selects the spacetime (Kerr, or
// the deformed metric through the metric-generic right-hand side). Every
// wave reads the host's stop request (if any) every 64 loop iterations and,
// once it is set, stores the photons it holds and leaves. The Kerr
// kernel takes 135 vector registers, three waves per SIMD; it would fit in
// 128 (four waves) without spilling, but measured slower that way (C2 +7%,
// far-field steady state +3%, 256-camera sweep -0.4%).
template <int PM = kPoleMonitor, int MET = GRAY_METRIC_KERR, bool STOP = false>
__global__ __launch_bounds__(kBlock) void k_integrate(IntArgs A)
{
    static_assert(MET == GRAY_METRIC_KERR || PM == kPoleMonitor,
                  "the deformed metric is integrated with the production pole treatment");
    using Space = typename std::conditional<MET == GRAY_METRIC_DEFORMED, DeformedSpin, Spin<double>>::type;
    const unsigned lane = threadIdx.x & (kWave - 1);
    const bool record_disk = (A.flags & GRAY_RECORD_DISK) != 0;
    const bool record_mark = A.mark != nullptr;
    const bool list_out = A.work_out != nullptr;
    const bool count_done = A.cam_done != nullptr;

    bool active = false;
    int64_t id = 0;
    Lane<GRAY_FP64> L;
    // (the launch-wide constants are set once, so that they stay uniform)
    StepConst<double, Space> K;
    K.step_frac = A.step_frac;
    K.xi_eps = A.xi_eps;
    K.euler_inv = A.euler_inv;
    const double resc = A.r_escape;
    double rcap = 0.0;
    int32_t nsteps = 0, ncall = 0, ne = 0, nr = 0, n64 = 0;
    bool hit = false;

    unsigned chunk_next = 0, chunk_end = 0;
    bool exhausted = false;
    // Two-ended queue (dense mode, where the launch order puts the photons
    // expected to take longest first): of the waves that share a SIMD, the
    // one in hardware slot 0 (HW_ID bits 3:0) issues first when several are
    // ready, and advances at close to the rate of a wave alone, while the
    // others get what is left (measured with two waves: about 2.4 vs 5 us
    // per step on the same work). Slot 0 therefore takes ids from the head
    // of the queue and the other slots from its tail, so the longest
    // photons run in the favoured slot.
    const bool from_tail = A.two_ended && (__builtin_amdgcn_s_getreg(4 | (3 << 11)) & 15u) != 0u;
    // Queue length: the length of the work list or of the launch order.
    const int64_t nq = (int64_t)__builtin_amdgcn_readfirstlane(*A.work_in_count);
    // A grab takes `grab` ids (a multiple of 64): large enough to keep the
    // single queue counter off the critical path, small enough that every wave
    // gets about four grabs.
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    int64_t rounds = nq / (waves * kQueueChunk * 4);
    rounds = rounds < 1 ? 1 : (rounds > kMaxGrab ? kMaxGrab : rounds);
    const unsigned grab = (unsigned)rounds * kQueueChunk;
    StopBook book;
    unsigned long long iters = 0;
    const bool watch = STOP && A.stop != nullptr;
    unsigned poll = 0;
    bool halt = false;
    // state, status, step count and counters of the photon that stops (or
    // pauses) in this lane
    auto store_photon = [&](int32_t st) {
        const ArgPointers PA = arg_pointers<1>();
        const int64_t S = A.stride;
        L.store(PA.x, PA.lo, S, id);
        glob(PA.status)[id] = st;
        glob(PA.steps)[id] = nsteps;
        if (PA.counters) {
            Column<int32_t> C(PA.counters, S, id);
            C.put(ne);
            C.next();
            C.put(nr);
            C.next();
            C.put(n64);
        }
    };

    for (;;) {
        if (watch && !halt && (poll++ & 63u) == 0u) halt = stop_requested();
        const uint64_t idle = ballot(!active);
        if (__popcll(idle) >= A.refill || idle == ~0ull) {
            if (chunk_next >= chunk_end && !exhausted)
                queue_grab(lane, from_tail, grab, nq, exhausted, chunk_next, chunk_end);
            const unsigned avail = chunk_end - chunk_next;
            if (avail > 0) {
                const unsigned rank = lane_rank(idle);
                const ArgPointers PA = arg_pointers<2>();
                const int64_t S = A.stride;
                if (!active && rank < avail) {
                    const unsigned q = chunk_next + rank;
                    id = (int64_t)glob(PA.work_in)[q];
                    if (id >= 0 && glob(PA.status)[id] == GRAY_RUNNING) {
                        L.load(PA.x, PA.lo, S, id);
                        const DevCam cm = PA.cams[glob(PA.cam)[id]];
                        if constexpr (MET == GRAY_METRIC_DEFORMED)
                            K.B = make_deformed(cm.a, cm.eps3);
                        else
                            K.B = make_spin(cm.a);
                        K.rbh = cm.rbh;
                        rcap = cm.rcap;
                        nsteps = glob(PA.steps)[id];
                        // a camera's own step budget counts against the
                        // call's: ncall reaches call_steps after it
                        ncall = cm.call_steps > 0 ? A.call_steps - cm.call_steps : 0;
                        ne = nr = n64 = 0;
                        if (PA.counters) {
                            Column<int32_t> C(PA.counters, S, id);
                            ne = C.get();
                            C.next();
                            nr = C.get();
                            C.next();
                            n64 = C.get();
                        }
                        hit = record_disk && glob(PA.disk)[id] != 0.0;
                        active = true;
                    }
                }
                const unsigned taken = __popcll(idle) < avail ? (unsigned)__popcll(idle) : avail;
                chunk_next += taken;
            }
            if (exhausted && chunk_next >= chunk_end && ballot(active) == 0ull) {
                book.finish(lane, list_out, iters);
                break;
            }
        }

        bool stop_now = false, keep = false;
        iters += ballot(active) != 0ull;
        if (active) {
            // Equatorial-crossing recorder and 2 r_bh mark of one accepted
            // step from xp to x, each a rare event tested wave-wide first.
            auto record = [&](const State<double> &xp, const State<double> &x) {
                const bool cross = record_disk && !hit && (xp.th - kHalfPi) * (x.th - kHalfPi) < 0.0;
                if (record_disk && __builtin_expect(any_lane(cross), 0) && cross) {
                    const double f = (kHalfPi - xp.th) / (x.th - xp.th);
                    const double rc = xp.r + f * (x.r - xp.r);
                    // recorder window of the photon's camera, read when needed
                    const DevCam &cw = GRAY_ARG(cams)[glob(GRAY_ARG(cam))[id]];
                    if (rc >= cw.disk_rmin && rc <= cw.disk_rmax) {
                        double E, Lz, Q, sx, cx;
                        sin_cos<true>(x.th, sx, cx);
                        conserved_sc(K.B.a, x, sx, cx, E, Lz, Q);
                        Column<double> D(GRAY_ARG(disk), A.stride, id);
                        D.put(rc);
                        D.next();
                        D.put(xp.ph + f * (x.ph - xp.ph));
                        D.next();
                        D.put(disk_redshift(K.B.a, rc, E, Lz));
                        hit = true;
                    }
                }
                const double rmark = K.rbh + K.rbh;
                const bool inward = xp.r >= rmark && x.r < rmark;
                if (record_mark && __builtin_expect(any_lane(inward), 0) && inward) {
                    const double v[8] = {xp.t, xp.r, xp.th, xp.ph, xp.kt, xp.kr, xp.kth, xp.kph};
                    Column<double> M(GRAY_ARG(mark), A.stride, id);
                    for (int k = 0; k < 8; ++k) {
                        M.put(v[k]);
                        if (k < 7) M.next();
                    }
                }
            };
            const int fl = rk4_step<PM>(K, L.x, L.s, L.c, record);
            const State<double> &x = L.x;
            int32_t st = GRAY_RUNNING;
            st = nsteps + (fl >= 0) >= A.max_steps ? GRAY_UNFINISHED : st;
            st = (x.r > resc && x.kr > 0.0) ? GRAY_ESCAPED : st;
            st = x.r < rcap ? GRAY_CAPTURED : st;
            st = (fl < 0 || !finite_state(x)) ? GRAY_NONFINITE : st;
            // counters after the step, taken with selects (no per-lane branch)
            const bool ok = fl >= 0;
            nsteps += ok;
            ncall += ok;
            ne += ok ? (fl & 1) : 0;
            nr += ok ? ((fl >> 1) & 1) : 0;
            // (after a stop request every photon pauses after its next step)
            const bool stop = halt || st != GRAY_RUNNING || (A.call_steps > 0 && ncall >= A.call_steps);
            if (__builtin_expect(any_lane(stop), 0) && stop) {
                store_photon(st);
                stop_now = true;
                keep = st == GRAY_RUNNING;
                active = false;
            }
        }
        book.account(stop_now, keep, id, lane, list_out, count_done);
    }
}

// ---------------------------------------------- compensated-float integrator
// The FP32C integrator. Each block has kBlock / kWave waves: all but the last
// run photons in float steps (rk4_step_f32) on the compensated state; the
// last runs FP64 steps. A photon goes over to FP64 for the rest of its path
// when it enters a zone the caller names (near the horizon, near a pole, at
// a radial turning point), or when the float step cannot decide the null
// monitor of eq. (4) (its proposal lies within float rounding of epsilon),
// and stays there: the counter of FP64 steps marks it, so a resumed call
// continues it in FP64 too. The float waves hand such photons to their
// block's FP64 wave through a small queue in LDS (state, step counts and
// recorder flag per slot), so neither kind of wave carries the other's
// code path or registers. While no photon waits for it, the FP64 wave runs
// float photons too, a few at a time (it takes new ones only while fewer
// than kHelperLimit photons wait, and returns to FP64 steps once its lanes
// are empty), so it is not idle where no photon needs FP64. Each phase is a
// loop of its own: no state is carried from one to the other.
constexpr int kHandCap = 128;            // hand-off slots per block
constexpr unsigned kFloatQuota = 64;     // slots the float waves may fill; the
                                         // rest takes the FP64 wave's own
                                         // hand-offs, so it never waits
constexpr unsigned kHelperLimit = 1;     // photons waiting, from which on the
                                         // FP64 wave takes no float work
constexpr int64_t kHelperPhotonsPerLane = 4;
// The FP64 wave in its float phase is the queue's only consumer and must
// never wait for a slot: it takes float work only while no slot is taken,
// so afterwards it adds at most kWave photons to the at most kFloatQuota
// the float waves may add.
static_assert(kHandCap >= (int)kFloatQuota + kWave, "the FP64 wave's own hand-offs always fit");
static_assert(kHelperLimit == 1, "the bound above assumes the helper refills only with no slot taken");

struct HandQueue {
    unsigned head;        // slots taken by the FP64 wave (monotonic)
    unsigned tail;        // slots reserved by the float waves (monotonic)
    unsigned float_done;  // float waves of the block that have exited
    unsigned halt;        // a float wave of the block has seen a stop request
    unsigned ready[kHandCap];
    int32_t id[kHandCap], nsteps[kHandCap], ncall[kHandCap], ne[kHandCap], nr[kHandCap], n64[kHandCap],
        hit[kHandCap];
    float hi[8][kHandCap], lo[8][kHandCap];
};

__device__ __forceinline__ unsigned lds_load(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_store(unsigned *p, unsigned v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Store one photon's counters and state at a stop (either loop).
__device__ __forceinline__ void c32_store(const Lane<GRAY_FP32C> &L, int64_t id, int32_t st, int32_t nsteps,
                                          int32_t ne, int32_t nr, int32_t n64, int64_t S)
{
    const ArgPointers PA = arg_pointers<1>();
    L.store(PA.x, PA.lo, S, id);
    glob(PA.status)[id] = st;
    glob(PA.steps)[id] = nsteps;
    Column<int32_t> C(PA.counters, S, id);
    C.put(ne);
    C.next();
    C.put(nr);
    C.next();
    C.put(n64);
}

// What a wave keeps from one phase to the next.
struct WaveCtx {
    bool exhausted = false;        // the global queue has nothing left for it
    bool halt = false;             // the host's stop request has been seen
    unsigned long long iters = 0;  // loop iterations with a stepping lane
    StopBook book;
};

// Float phase: the persistent loop of k_integrate with the float step. The
// float waves run it once, for their whole life; the FP64 wave runs it as a
// helper (HELPER): it takes ids only as many as it has idle lanes and only
// while fewer than kHelperLimit photons wait for FP64, and the phase ends
// once its lanes are empty.
template <bool HELPER, bool STOP>
__device__ __forceinline__ void c32_float_phase(const IntArgs &A, HandQueue &Q, unsigned nfloat_waves, WaveCtx &W)
{
    const unsigned lane = threadIdx.x & (kWave - 1);
    const bool record_disk = (A.flags & GRAY_RECORD_DISK) != 0;
    const bool record_mark = A.mark != nullptr;
    const bool list_out = A.work_out != nullptr;
    const bool count_done = A.cam_done != nullptr;

    bool active = false, pending = false;
    int64_t id = 0;
    Lane<GRAY_FP32C> L;
    // (the launch-wide constants are set once, so that they stay uniform)
    StepConst<float> Kf;
    Kf.step_frac = (float)A.step_frac;
    Kf.xi_eps = (float)A.xi_eps;
    Kf.euler_inv = (float)A.euler_inv;
    FloatHorizon Hf{};
    float r64 = 0.0f, rcap_f = 0.0f, rmark_f = 0.0f, rband_f = 0.0f;
    const float pole_f = (float)A.fp64_pole, turn_f = (float)A.fp64_turn;
    const float resc_f = (float)(A.r_escape * (1.0 - 1e-6));
    double rcap = 0.0;
    int32_t nsteps = 0, ncall = 0, ne = 0, nr = 0, n64 = 0;
    bool hit = false;

    unsigned chunk_next = 0, chunk_end = 0;
    bool &exhausted = W.exhausted;
    // (the helper takes from the tail, where the launch order puts the
    // photons expected to be shortest, so its phases end soon)
    const bool from_tail =
        A.two_ended && (HELPER || (__builtin_amdgcn_s_getreg(4 | (3 << 11)) & 15u) != 0u);
    const int64_t nq = (int64_t)__builtin_amdgcn_readfirstlane(*A.work_in_count);
    const int64_t waves = (int64_t)gridDim.x * nfloat_waves;
    int64_t rounds = nq / (waves * kQueueChunk * 4);
    rounds = rounds < 1 ? 1 : (rounds > kMaxGrab ? kMaxGrab : rounds);
    StopBook &book = W.book;
    unsigned long long &iters = W.iters;
    const bool watch = STOP && A.stop != nullptr;
    unsigned poll = 0;
    bool &halt = W.halt;

    for (;;) {
        if (watch && !halt && (poll++ & 63u) == 0u) {
            halt = stop_requested();
            if (halt) {
                if (HELPER) exhausted = true;   // the FP64 wave takes no more float work
                else if (lane == 0) lds_store(&Q.halt, 1u);   // for the block's FP64 wave
            }
        }
        const uint64_t idle = ballot(!active);
        // the helper takes float work only while few photons wait for it
        const bool may_take = !HELPER || lds_load(&Q.tail) - lds_load(&Q.head) < kHelperLimit;
        if (HELPER && idle == ~0ull && (!may_take || exhausted)) break;
        if (__popcll(idle) >= A.refill || idle == ~0ull) {
            // a helper grabs as many ids as it has idle lanes, so it leaves
            // no ids behind when its phase ends
            const unsigned grab = HELPER ? (unsigned)__popcll(idle) : (unsigned)rounds * kQueueChunk;
            if (chunk_next >= chunk_end && !exhausted && may_take)
                queue_grab(lane, from_tail, grab, nq, exhausted, chunk_next, chunk_end);
            const unsigned avail = chunk_end - chunk_next;
            if (avail > 0) {
                const unsigned rank = lane_rank(idle);
                const ArgPointers PA = arg_pointers<2>();
                const int64_t S = A.stride;
                if (!active && rank < avail) {
                    const unsigned q = chunk_next + rank;
                    id = (int64_t)glob(PA.work_in)[q];
                    if (id >= 0 && glob(PA.status)[id] == GRAY_RUNNING) {
                        L.load(PA.x, PA.lo, S, id);
                        const DevCam cm = PA.cams[glob(PA.cam)[id]];
                        Kf.B = make_spin((float)cm.a);
                        Kf.rbh = (float)cm.rbh;
                        Hf = make_float_horizon(cm.a);
                        r64 = (float)(cm.rbh * (1.0 + A.fp64_horizon));
                        rcap_f = (float)(cm.rcap * (1.0 + 1e-6));
                        rmark_f = (float)(2.0 * cm.rbh);
                        rband_f = (float)(2.0 * cm.rbh * (1.0 + 2.0 * A.step_frac));
                        rcap = cm.rcap;
                        nsteps = glob(PA.steps)[id];
                        // a camera's own step budget counts against the
                        // call's: ncall reaches call_steps after it
                        ncall = cm.call_steps > 0 ? A.call_steps - cm.call_steps : 0;
                        Column<int32_t> C(PA.counters, S, id);
                        ne = C.get();
                        C.next();
                        nr = C.get();
                        C.next();
                        n64 = C.get();
                        hit = record_disk && glob(PA.disk)[id] != 0.0;
                        active = true;
                        pending = n64 > 0;   // it continues in FP64
                    }
                }
                const unsigned taken = __popcll(idle) < avail ? (unsigned)__popcll(idle) : avail;
                chunk_next += taken;
            }
            if (!HELPER && exhausted && chunk_next >= chunk_end && ballot(active) == 0ull) {
                book.finish(lane, list_out, iters);
                if (lane == 0)
                    __hip_atomic_fetch_add(&Q.float_done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                break;
            }
        }

        bool stop_now = false, keep = false;
        iters += ballot(active && !pending) != 0ull;
        if (active && !pending) {
            auto &F = L;
            const bool need64 = F.hi.r < r64 || F.s < pole_f || fabsf(F.hi.kr) < turn_f * fabsf(F.hi.kt);
            // A photon at r in [2 r_bh, 2 r_bh (1 + 2 Delta)) may fall below
            // 2 r_bh in this step (a step moves r by at most about Delta r):
            // its state is kept as the mark before a float step.
            const bool band = record_mark && !need64 && F.hi.r >= rmark_f && F.hi.r < rband_f;
            if (__builtin_expect(any_lane(band), 0) && band) {
                const State<double> xm = F.value();
                const double v[8] = {xm.t, xm.r, xm.th, xm.ph, xm.kt, xm.kr, xm.kth, xm.kph};
                Column<double> M(GRAY_ARG(mark), A.stride, id);
                for (int k = 0; k < 8; ++k) {
                    M.put(v[k]);
                    if (k < 7) M.next();
                }
            }
            const float pth = F.hi.th, pr = F.hi.r, pph = F.hi.ph;
            int fl = -2;
            if (any_lane(!need64) && !need64) fl = rk4_step_f32(Kf, Hf, F.hi, F.lo, F.s, F.c);
            pending = fl == -2;
            if (!pending) {
                if (record_disk && fl >= 0) {
                    const bool cross = !hit && (pth - (float)kHalfPi) * (F.hi.th - (float)kHalfPi) <= 0.0f;
                    if (__builtin_expect(any_lane(cross), 0) && cross) {
                        const State<double> x = F.value();
                        const double ppth = pth, ppr = pr, ppph = pph;
                        const double f = (kHalfPi - ppth) / (x.th - ppth);
                        const double rc = ppr + f * (x.r - ppr);
                        const DevCam &cw = GRAY_ARG(cams)[glob(GRAY_ARG(cam))[id]];
                        if (rc >= cw.disk_rmin && rc <= cw.disk_rmax) {
                            double E, Lz, Qc, sx, cx;
                            sin_cos<false>(x.th, sx, cx);
                            conserved_sc(cw.a, x, sx, cx, E, Lz, Qc);
                            Column<double> D(GRAY_ARG(disk), A.stride, id);
                            D.put(rc);
                            D.next();
                            D.put(ppph + f * (x.ph - ppph));
                            D.next();
                            D.put(disk_redshift(cw.a, rc, E, Lz));
                            hit = true;
                        }
                    }
                }
                // Termination tests on the float high words, exact (hi + lo
                // in FP64) only for photons within a relative 1e-6 of a threshold.
                int32_t st = GRAY_RUNNING;
                st = nsteps + (fl >= 0) >= A.max_steps ? GRAY_UNFINISHED : st;
                const bool near = F.hi.r < rcap_f || (F.hi.r > resc_f && F.hi.kr >= 0.0f);
                if (__builtin_expect(any_lane(near), 0) && near) {
                    const double xr = (double)F.hi.r + (double)F.lo.r;
                    const double xkr = (double)F.hi.kr + (double)F.lo.kr;
                    st = (xr > A.r_escape && xkr > 0.0) ? GRAY_ESCAPED : st;
                    st = xr < rcap ? GRAY_CAPTURED : st;
                }
                const bool finite = __builtin_isfinite(F.hi.t) && __builtin_isfinite(F.hi.r) &&
                                    __builtin_isfinite(F.hi.th) && __builtin_isfinite(F.hi.ph) &&
                                    __builtin_isfinite(F.hi.kt) && __builtin_isfinite(F.hi.kr) &&
                                    __builtin_isfinite(F.hi.kth) && __builtin_isfinite(F.hi.kph);
                st = (fl < 0 || !finite) ? GRAY_NONFINITE : st;
                const bool ok = fl >= 0;
                nsteps += ok;
                ncall += ok;
                ne += ok ? (fl & 1) : 0;
                nr += ok ? ((fl >> 1) & 1) : 0;
                // (after a stop request every photon pauses after its next step)
                const bool stop = halt || st != GRAY_RUNNING || (A.call_steps > 0 && ncall >= A.call_steps);
                if (__builtin_expect(any_lane(stop), 0) && stop) {
                    c32_store(L, id, st, nsteps, ne, nr, n64, A.stride);
                    stop_now = true;
                    keep = st == GRAY_RUNNING;
                    active = false;
                }
            }
        }
        // After a stop request a photon that needs FP64 is stored as it
        // stands (its step not taken) instead of handed over.
        if (__builtin_expect(halt, 0) && active && pending) {
            c32_store(L, id, GRAY_RUNNING, nsteps, ne, nr, n64, A.stride);
            stop_now = keep = true;
            active = pending = false;
        }
        book.account(stop_now, keep, id, lane, list_out, count_done);

        // Photons that continue in FP64 go to the block's FP64 wave: reserve
        // slots (all of them or none this iteration, by compare-and-swap on
        // the reservation counter), fill them, then publish each slot.
        const uint64_t pm = ballot(active && pending);
        if (__builtin_expect(pm != 0ull, 0)) {
            const unsigned k = (unsigned)__popcll(pm);
            unsigned base = 0, ok = 0;
            if (lane == 0) {
                const unsigned t = lds_load(&Q.tail);
                const unsigned h = lds_load(&Q.head);
                if (t - h + k <= (HELPER ? (unsigned)kHandCap : kFloatQuota) && atomicCAS(&Q.tail, t, t + k) == t) {
                    base = t;
                    ok = 1;
                }
            }
            ok = __builtin_amdgcn_readfirstlane(ok);
            if (ok) {
                base = __builtin_amdgcn_readfirstlane(base);
                if (active && pending) {
                    const unsigned s = (base + lane_rank(pm)) % kHandCap;
                    Q.id[s] = (int32_t)id;
                    Q.nsteps[s] = nsteps;
                    Q.ncall[s] = ncall;
                    Q.ne[s] = ne;
                    Q.nr[s] = nr;
                    Q.n64[s] = n64;
                    Q.hit[s] = hit;
                    const float *h = &L.hi.t, *l = &L.lo.t;
                    for (int c = 0; c < 8; ++c) {
                        Q.hi[c][s] = h[c];
                        Q.lo[c][s] = l[c];
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    lds_store(&Q.ready[s], 1u);
                    active = false;
                    pending = false;
                }
            } else if (pm == ballot(active)) {
                __builtin_amdgcn_s_sleep(2);   // every busy lane waits for a slot
            }
        }
    }
}

// FP64 phase of a block's FP64 wave: photons handed over by the block's
// waves, FP64 steps on the compensated pair until they stop. Each step
// rounds the state to 48-bit significands, which the float pair holds
// exactly, and takes its sin/cos there, so a resumed call (which rebuilds
// the state from the pair) continues bit for bit. Returns true when the wave
// is done (the float waves of its block have exited and every handed-over
// photon has stopped or paused), false when it has nothing to do but the
// global queue may still hold float work. Once nothing more can arrive the
// wave finishes its photons in a loop of their steps alone: without the
// queue's code around it the register allocator keeps the step's values in
// place (in the polling loop it splits them around the hand-over, about 45
// register copies per step), which is what a launch's last photons run.
template <bool STOP>
__device__ __forceinline__ bool c32_fp64_phase(const IntArgs &A, HandQueue &Q, unsigned nfloat_waves, WaveCtx &W)
{
    const unsigned lane = threadIdx.x & (kWave - 1);
    const bool record_disk = (A.flags & GRAY_RECORD_DISK) != 0;
    const bool record_mark = A.mark != nullptr;
    const bool list_out = A.work_out != nullptr;
    const bool count_done = A.cam_done != nullptr;

    bool active = false;
    int64_t id = 0;
    State<double> x{};   // always a sum hi + lo of two floats
    double s64 = 0.0, c64 = 1.0;   // sin and cos of x.th
    // (the launch-wide constants are set once, so that they stay uniform)
    StepConst<double, Spin<double>> K;
    K.step_frac = A.step_frac;
    K.xi_eps = A.xi_eps;
    K.euler_inv = A.euler_inv;
    double rcap = 0.0;
    int32_t nsteps = 0, ncall = 0, ne = 0, nr = 0, n64 = 0;
    bool hit = false;
    StopBook &book = W.book;
    unsigned long long &iters = W.iters;
    // The queue is closed once the block's float waves have exited (every
    // slot they reserved is then published) and every slot has been taken:
    // nothing more can arrive, and the wave leaves the polling loop for a
    // loop of its own photons alone.
    unsigned tick = 0;

    // One step of every active lane; `halt` stores each after its step.
    auto advance = [&](bool halt) __attribute__((always_inline)) {
        bool stop_now = false, keep = false;
        iters += ballot(active) != 0ull;
        if (active) {
            auto record_disk_event = [&](double pth, double pr, double pph, const State<double> &x) {
                const bool cross = record_disk && !hit && (pth - kHalfPi) * (x.th - kHalfPi) < 0.0;
                if (record_disk && __builtin_expect(any_lane(cross), 0) && cross) {
                    const double f = (kHalfPi - pth) / (x.th - pth);
                    const double rc = pr + f * (x.r - pr);
                    const DevCam &cw = GRAY_ARG(cams)[glob(GRAY_ARG(cam))[id]];
                    if (rc >= cw.disk_rmin && rc <= cw.disk_rmax) {
                        double E, Lz, Qc, sx, cx;
                        sin_cos<false>(x.th, sx, cx);
                        conserved_sc(K.B.a, x, sx, cx, E, Lz, Qc);
                        Column<double> D(GRAY_ARG(disk), A.stride, id);
                        D.put(rc);
                        D.next();
                        D.put(pph + f * (x.ph - pph));
                        D.next();
                        D.put(disk_redshift(K.B.a, rc, E, Lz));
                        hit = true;
                    }
                }
            };
            auto record = [&](const State<double> &xp, const State<double> &x) {
                record_disk_event(xp.th, xp.r, xp.ph, x);
                const double rmark = K.rbh + K.rbh;
                const bool inward = xp.r >= rmark && x.r < rmark;
                if (record_mark && __builtin_expect(any_lane(inward), 0) && inward) {
                    const double v[8] = {xp.t, xp.r, xp.th, xp.ph, xp.kt, xp.kr, xp.kth, xp.kph};
                    Column<double> M(GRAY_ARG(mark), A.stride, id);
                    for (int k = 0; k < 8; ++k) {
                        M.put(v[k]);
                        if (k < 7) M.next();
                    }
                }
            };
            // (the step rounds the state to the float pair it is stored as)
            const int fl = rk4_step<kPoleMonitor, true, true>(K, x, s64, c64, record);
            const State<double> &xr = x;
            int32_t st = GRAY_RUNNING;
            st = nsteps + (fl >= 0) >= A.max_steps ? GRAY_UNFINISHED : st;
            st = (xr.r > A.r_escape && xr.kr > 0.0) ? GRAY_ESCAPED : st;
            st = xr.r < rcap ? GRAY_CAPTURED : st;
            st = (fl < 0 || !finite_state(xr)) ? GRAY_NONFINITE : st;
            const bool ok = fl >= 0;
            nsteps += ok;
            ncall += ok;
            ne += ok ? (fl & 1) : 0;
            nr += ok ? ((fl >> 1) & 1) : 0;
            n64 += ok;
            const bool stop = halt || st != GRAY_RUNNING || (A.call_steps > 0 && ncall >= A.call_steps);
            if (__builtin_expect(any_lane(stop), 0) && stop) {
                Lane<GRAY_FP32C> P;
                P.split(x);
                c32_store(P, id, st, nsteps, ne, nr, n64, A.stride);
                stop_now = true;
                keep = st == GRAY_RUNNING;
                active = false;
            }
        }
        book.account(stop_now, keep, id, lane, list_out, count_done);
    };

    for (;;) {
        const uint64_t idle = ballot(!active);
        // Poll while the queue may still receive photons: whenever every lane
        // or a quarter of the lanes are idle, otherwise every fourth
        // iteration (a wave with few photons left spends little of its step
        // on the queue's loads).
        ++tick;
        if (idle && (idle == ~0ull || __popcll(idle) >= kWave / 4 || (tick & 3u) == 0u)) {
            const unsigned done = __hip_atomic_load(&Q.float_done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            // after a stop request (seen by the block's float waves) this wave
            // takes no more float work
            if (STOP && __builtin_amdgcn_readfirstlane(lds_load(&Q.halt)) != 0u) W.exhausted = true;
            const unsigned h = __builtin_amdgcn_readfirstlane(lds_load(&Q.head));
            const unsigned t = __builtin_amdgcn_readfirstlane(lds_load(&Q.tail));
            // slots h, h + 1, ... that are published, as many as lanes are idle
            const bool rdy = lane < t - h && lds_load(&Q.ready[(h + lane) % kHandCap]) != 0u;
            const uint64_t rm = ballot(rdy);
            unsigned c = (unsigned)__ffsll((long long)~rm) - 1u;   // published prefix
            c = c < (unsigned)__popcll(idle) ? c : (unsigned)__popcll(idle);
            if (c > 0) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const unsigned rank = lane_rank(idle);
                const bool took = !active && rank < c;
                if (took) {
                    const unsigned s = (h + rank) % kHandCap;
                    id = Q.id[s];
                    nsteps = Q.nsteps[s];
                    ncall = Q.ncall[s];
                    ne = Q.ne[s];
                    nr = Q.nr[s];
                    n64 = Q.n64[s];
                    hit = Q.hit[s] != 0;
                    double *xp = &x.t;
                    for (int k = 0; k < 8; ++k) xp[k] = (double)Q.hi[k][s] + (double)Q.lo[k][s];
                    sin_cos<true>(x.th, s64, c64);
                    const DevCam cm = GRAY_ARG(cams)[glob(GRAY_ARG(cam))[id]];
                    K.B = make_spin(cm.a);
                    K.rbh = cm.rbh;
                    rcap = cm.rcap;
                    active = true;
                }
                // every read of the taken slots is done before they are freed
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (took) lds_store(&Q.ready[(h + rank) % kHandCap], 0u);
                if (lane == 0) lds_store(&Q.head, h + c);
            } else {
                const bool closed = done == nfloat_waves && h == t;
                if (idle == ~0ull) {
                    if (closed) return true;
                    if (!W.exhausted && A.helper) return false;
                    __builtin_amdgcn_s_sleep(2);
                    continue;
                }
                if (closed) break;
            }
        }

        advance(false);
    }

    // Tail: the queue is closed and only the wave's own photons remain. Here
    // the wave reads the stop request itself (the flag of its block's float
    // waves, then the host's every 64 iterations).
    const bool watch = STOP && A.stop != nullptr;
    bool halt = STOP && (W.halt || __builtin_amdgcn_readfirstlane(lds_load(&Q.halt)) != 0u);
    unsigned poll = 0;
    while (ballot(active) != 0ull) {
        if (watch && !halt && (poll++ & 63u) == 0u) halt = stop_requested();
        advance(halt);
    }
    return true;
}

// Four waves per SIMD (at most 128 vector registers). The float loop fits;
// the FP64 loop keeps a few values in scratch memory, which costs its steps
// less than the fourth wave gains the float ones (against three waves per
// SIMD and no spills in its steps: far-field steady state -12%, 2048^2 of the
// 4096^2 recorder workload -14%, 256-camera sweep -9%, the 512^2 edge-on grid,
// bound by one photon in the FP64 loop, +3%).
//
// BLK: threads per block, each block one FP64 wave and BLK / 64 - 1 float
// waves. Where the launch is bound by throughput, 512: a block of 448 float
// lanes gives its FP64 wave about twice the photons that 192 do, and the
// FP64 steps (a few percent of the steps there) cost about half as many wave
// instructions (256-camera sweep -7%, 2048^2 of the 4096^2 recorder workload
// -5%, far-field steady state unchanged). Where the launch is bound by its
// longest photons, 256: the 512^2 edge-on grid takes a fifth of its steps in
// FP64, which one wave per 448 float lanes cannot keep up with (+12-20%).
template <bool STOP = false, int BLK = kBlock>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(4))) void k_integrate_c32(IntArgs A)
{
    static_assert(BLK % kWave == 0 && BLK / kWave >= 2 && BLK >= kHandCap, "one FP64 wave, one float wave at least");
    __shared__ HandQueue Q;
    constexpr unsigned kWaves = BLK / kWave;
    if (threadIdx.x < (unsigned)kHandCap) Q.ready[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        Q.head = 0u;
        Q.tail = 0u;
        Q.float_done = 0u;
        Q.halt = 0u;
    }
    __syncthreads();
    const unsigned lane = threadIdx.x & (kWave - 1);
    WaveCtx W;
    if (threadIdx.x / kWave == kWaves - 1) {
        while (!c32_fp64_phase<STOP>(A, Q, kWaves - 1, W) && A.helper)
            c32_float_phase<true, STOP>(A, Q, kWaves - 1, W);
        W.book.finish(lane, A.work_out != nullptr, W.iters);
    } else {
        c32_float_phase<false, STOP>(A, Q, kWaves - 1, W);
    }
}

// ------------------------------------------------------------- classification
struct ClassArgs {
    const void *x, *lo;
    const int32_t *status;
    const double *mark;
    int8_t *flag;
    double *xf, *cons;
    int32_t *counts;
    int64_t stride;
    int32_t precision, pad;
    CamChunk ch;
};

__global__ __launch_bounds__(kBlock) void k_zero_i32(int32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Work-list classification: flags and per-camera status counts of the listed
// photons only (grid-stride over a list whose length is on the device).
__global__ __launch_bounds__(kBlock) void k_classify_list(const int32_t *list, const unsigned *count,
                                                          const int32_t *status, const int32_t *cam,
                                                          int8_t *flag, int32_t *counts, int32_t ncam)
{
    const int64_t n = (int64_t)__builtin_amdgcn_readfirstlane(*count);
    const unsigned lane = threadIdx.x & (kWave - 1);
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const int64_t i = list[j];
        if (i < 0) continue;
        const int32_t st = status[i];
        flag[i] = (int8_t)st;
        if (!counts) continue;
        const int sb = (st >= 0 && st < 5) ? st : 4;
        const int32_t c = cam[i];
        const int32_t c0 = __builtin_amdgcn_readfirstlane(c);
        if (ballot(c != c0) == 0ull) {
            if (c0 < 0 || c0 >= ncam) continue;
            const uint64_t act = ballot(true);
            for (int k = 0; k < 5; ++k) {
                const uint64_t m = ballot(sb == k);
                if (m && lane == (unsigned)(__ffsll((long long)act) - 1))
                    atomicAdd(&counts[c0 * 5 + k], (int)__popcll(m));
            }
        } else if (c >= 0 && c < ncam) {
            atomicAdd(&counts[c * 5 + sb], 1);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_classify(ClassArgs A)
{
    const int64_t i = A.ch.lo + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.ch.hi) return;
    const int k = find_camera(A.ch, i);
    if (k < 0) return;
    const CamArg &c = A.ch.c[k];
    const int64_t S = A.stride;
    const int32_t st = A.status[i];
    A.flag[i] = (int8_t)st;
    if (A.counts) {
        // One atomic per wave and status when the wave's photons share a
        // camera (the common case), else one per photon.
        const int sb = (st >= 0 && st < 5) ? st : 4;
        const int c0 = __builtin_amdgcn_readfirstlane(c.index);
        if (ballot(c.index != c0) == 0ull) {
            const uint64_t act = ballot(true);
            const unsigned lane = threadIdx.x & (kWave - 1);
            for (int k = 0; k < 5; ++k) {
                const uint64_t m = ballot(sb == k);
                if (m && lane == (unsigned)(__ffsll((long long)act) - 1))
                    atomicAdd(&A.counts[c0 * 5 + k], (int)__popcll(m));
            }
        } else {
            atomicAdd(&A.counts[c.index * 5 + sb], 1);
        }
    }

    State<double> xf;
    double v[8];
    if (A.precision == GRAY_FP64) {
        const double *X = (const double *)A.x;
        for (int j = 0; j < 8; ++j) v[j] = X[j * S + i];
    } else {
        const float *H = (const float *)A.x, *L = (const float *)A.lo;
        for (int j = 0; j < 8; ++j) v[j] = (double)H[j * S + i] + (double)L[j * S + i];
    }
    xf.t = v[0]; xf.r = v[1]; xf.th = v[2]; xf.ph = v[3];
    xf.kt = v[4]; xf.kr = v[5]; xf.kth = v[6]; xf.kph = v[7];
    if (A.xf)
        for (int j = 0; j < 8; ++j) A.xf[j * S + i] = v[j];
    if (A.cons) {
        double alpha, beta;
        pixel_of(c, i, alpha, beta);
        State<double> x0;
        const bool deformed = c.metric == GRAY_METRIC_DEFORMED;
        camera_state(c.a, c.r_obs, c.incl, alpha, beta, x0, c.eps3, deformed);
        double E0, L0, Q0, E, L, Q;
        conserved_in(c.a, c.eps3, deformed, x0, E0, L0, Q0);
        conserved_in(c.a, c.eps3, deformed, xf, E, L, Q);
        State<double> xd = xf;
        if (st == GRAY_CAPTURED && A.mark && A.mark[1 * S + i] > 0.0) {
            xd.t = A.mark[0 * S + i]; xd.r = A.mark[1 * S + i];
            xd.th = A.mark[2 * S + i]; xd.ph = A.mark[3 * S + i];
            xd.kt = A.mark[4 * S + i]; xd.kr = A.mark[5 * S + i];
            xd.kth = A.mark[6 * S + i]; xd.kph = A.mark[7 * S + i];
        }
        double Ed, Ld, Qd;
        conserved_in(c.a, c.eps3, deformed, xd, Ed, Ld, Qd);
        double *C = A.cons;
        C[0 * S + i] = E0;
        C[1 * S + i] = L0;
        C[2 * S + i] = Q0;
        C[3 * S + i] = E;
        C[4 * S + i] = L;
        C[5 * S + i] = Q;
        C[6 * S + i] = fabs(Ed / E0 - 1.0);
        C[7 * S + i] = fabs(Ld - L0) / (fabs(L0) + fabs(E0));
        C[8 * S + i] = fabs(Qd - Q0) / (fabs(Q0) + L0 * L0 + E0 * E0);
    }
}

// ------------------------------------------------------------- host helpers
static int validate_params(const gray_params *p)
{
    if (!p) return GRAY_EINVAL;
    if (!(p->step_frac > 0.0 && std::isfinite(p->step_frac))) return GRAY_EINVAL;
    if (!(p->horizon_eps > 0.0 && std::isfinite(p->horizon_eps))) return GRAY_EINVAL;
    if (!(p->r_escape > 0.0 && std::isfinite(p->r_escape))) return GRAY_EINVAL;
    if (!(p->xi_eps > 0.0)) return GRAY_EINVAL;
    if (!(p->euler_div >= 1.0 && std::isfinite(p->euler_div))) return GRAY_EINVAL;
    if (p->max_steps < 1 || p->call_steps < 0) return GRAY_EINVAL;
    if (p->precision != GRAY_FP64 && p->precision != GRAY_FP32C) return GRAY_EINVAL;
    if (p->flags & ~(GRAY_RECORD_DISK | GRAY_SLOTS | GRAY_WORKLIST)) return GRAY_EINVAL;
    if (!(p->fp64_horizon >= 0.0 && std::isfinite(p->fp64_horizon))) return GRAY_EINVAL;
    if (!(p->fp64_pole >= 0.0 && std::isfinite(p->fp64_pole))) return GRAY_EINVAL;
    if (!(p->fp64_turn >= 0.0 && std::isfinite(p->fp64_turn))) return GRAY_EINVAL;
    if (p->pole_mode != GRAY_POLE_MONITOR && p->pole_mode != GRAY_POLE_EULER_CROSSING &&
        p->pole_mode != GRAY_POLE_NONE)
        return GRAY_EINVAL;
    if (p->precision == GRAY_FP32C && p->pole_mode != GRAY_POLE_MONITOR) return GRAY_EUNSUPPORTED;
    if (p->flags & GRAY_RECORD_DISK) {
        if (!(p->disk_rmax > 0.0) || std::isnan(p->disk_rmin)) return GRAY_EINVAL;
    }
    return GRAY_OK;
}

static bool camera_physical_ok(const gray_camera &c)
{
    if (c.kind != GRAY_CAMERA_GRID && c.kind != GRAY_CAMERA_POLAR) return false;
    if (!(c.a >= 0.0 && c.a < 1.0)) return false;
    if (c.metric == GRAY_METRIC_KERR) {
        if (c.deform != 0.0) return false;
    } else if (c.metric == GRAY_METRIC_DEFORMED) {
        // regular outside the Kerr horizon: 1 + h > 0 and Delta + a^2 sin^2 h > 0
        if (!std::isfinite(c.deform)) return false;
        if (!(c.deform >= 0.0 || (c.a == 0.0 && c.deform > -8.0))) return false;
    } else {
        return false;
    }
    if (!(c.r_obs > horizon_radius(c.a) && std::isfinite(c.r_obs))) return false;
    if (!(c.incl >= 0.0 && c.incl <= kPi)) return false;
    if (c.call_steps < 0) return false;
    return std::isfinite(c.alpha_lo) && std::isfinite(c.alpha_hi) && std::isfinite(c.beta_lo) &&
           std::isfinite(c.beta_hi);
}

// Dense mode: cameras tile [0, n) in order. Slot mode: disjoint ranges inside
// [0, n) in any order, empty slots allowed.
static int validate_cameras(const gray_camera *cams, int32_t ncam, int64_t n, uint32_t flags)
{
    if (!cams || ncam < 1) return GRAY_EINVAL;
    if (flags & GRAY_SLOTS) {
        std::vector<std::pair<int64_t, int64_t>> r;
        r.reserve(ncam);
        for (int32_t k = 0; k < ncam; ++k) {
            const gray_camera &c = cams[k];
            if (c.nx < 0 || c.ny < 0) return GRAY_EINVAL;
            const int64_t m = (int64_t)c.nx * c.ny;
            if (m == 0) continue;
            if (!camera_physical_ok(c)) return GRAY_EINVAL;
            if (c.first < 0 || c.first + m > n) return GRAY_EINVAL;
            r.emplace_back(c.first, c.first + m);
        }
        std::sort(r.begin(), r.end());
        for (size_t k = 1; k < r.size(); ++k)
            if (r[k].first < r[k - 1].second) return GRAY_EINVAL;
        return GRAY_OK;
    }
    int64_t next = 0;
    for (int32_t k = 0; k < ncam; ++k) {
        const gray_camera &c = cams[k];
        if (!camera_physical_ok(c)) return GRAY_EINVAL;
        if (c.nx < 1 || c.ny < 1) return GRAY_EINVAL;
        if (c.first != next) return GRAY_EINVAL;
        next += (int64_t)c.nx * c.ny;
        if (next > n) return GRAY_EINVAL;
    }
    return next == n ? GRAY_OK : GRAY_EINVAL;
}

// The spacetime of a call: every camera (every non-empty slot) must use the
// same metric kind; the deformed metric is served in FP64 with the
// production pole treatment and without the disk recorder. Call after
// validate_cameras.
static int call_metric(const gray_camera *cams, int32_t ncam, const gray_params *p, int *metric)
{
    int m = -1;
    for (int32_t k = 0; k < ncam; ++k) {
        if ((int64_t)cams[k].nx * cams[k].ny == 0) continue;
        if (m < 0) m = cams[k].metric;
        else if (cams[k].metric != m) return GRAY_EUNSUPPORTED;
    }
    if (m < 0) m = GRAY_METRIC_KERR;
    if (m == GRAY_METRIC_DEFORMED &&
        (p->precision != GRAY_FP64 || p->pole_mode != GRAY_POLE_MONITOR || (p->flags & GRAY_RECORD_DISK)))
        return GRAY_EUNSUPPORTED;
    *metric = m;
    return GRAY_OK;
}

static int validate_state(const gray_state *s, const gray_params *p)
{
    if (!s) return GRAY_EINVAL;
    if (s->n < 0 || s->n > GRAY_MAX_PHOTONS) return GRAY_EINVAL;
    if (s->n == 0) return GRAY_OK;
    if (s->stride < s->n || s->stride % kWave != 0) return GRAY_EINVAL;
    if (!s->x || !s->status || !s->steps || !s->cam) return GRAY_EINVAL;
    if (p->precision == GRAY_FP32C && !s->lo) return GRAY_EINVAL;
    if (p->precision == GRAY_FP64 && s->lo) return GRAY_EINVAL;
    if ((p->flags & GRAY_RECORD_DISK) && !s->disk) return GRAY_EINVAL;
    const bool wl = (p->flags & GRAY_WORKLIST) != 0;
    if (wl != (s->work_in && s->work_out && s->work_in_count && s->work_out_count)) return GRAY_EINVAL;
    if (!wl && (s->work_in || s->work_out || s->work_in_count || s->work_out_count)) return GRAY_EINVAL;
    return GRAY_OK;
}

// Chunk of up to kCamChunk cameras as a kernel argument; in slot mode empty
// slots are left out. Returns false when the chunk covers no photon.
static bool fill_chunk(const gray_camera *cams, int32_t k0, int32_t cnt, bool slots, CamChunk &ch)
{
    memset(&ch, 0, sizeof ch);
    ch.sparse = slots ? 1 : 0;
    int64_t lo = INT64_MAX, hi = 0;
    for (int32_t j = 0; j < cnt; ++j) {
        const gray_camera &c = cams[k0 + j];
        const int64_t m = (int64_t)c.nx * c.ny;
        if (m == 0) continue;
        CamArg &o = ch.c[ch.count++];
        o.a = c.a;
        o.r_obs = c.r_obs;
        o.incl = c.incl;
        o.alo = c.alpha_lo;
        o.ahi = c.alpha_hi;
        o.blo = c.beta_lo;
        o.bhi = c.beta_hi;
        o.first = c.first;
        o.nx = c.nx;
        o.ny = c.ny;
        o.index = k0 + j;
        o.kind = c.kind;
        o.metric = c.metric;
        o.eps3 = c.deform;
        lo = std::min(lo, c.first);
        hi = std::max(hi, c.first + m);
    }
    ch.lo = lo;
    ch.hi = hi;
    return ch.count > 0;
}

// Integrator variants: FP64 with each pole treatment, FP32C (production
// treatment only), FP64 in the deformed metric (production treatment only);
// each in a second build that honours gray_state::stop (its test costs the
// loop 1-4%, so a call without a stop flag runs the build without it).
constexpr int kVariants = 6;
// FP32C block shapes (variant 1 and kVariantC32Wide)
constexpr int kBlockC32Wide = 512;
constexpr int kVariantC32Wide = 5;

template <bool STOP>
static void variant_kernels(const void *k[kVariants])
{
    k[0] = (const void *)k_integrate<kPoleMonitor, GRAY_METRIC_KERR, STOP>;
    k[1] = (const void *)k_integrate_c32<STOP>;
    k[2] = (const void *)k_integrate<kPoleEulerCrossing, GRAY_METRIC_KERR, STOP>;
    k[3] = (const void *)k_integrate<kPoleNone, GRAY_METRIC_KERR, STOP>;
    k[4] = (const void *)k_integrate<kPoleMonitor, GRAY_METRIC_DEFORMED, STOP>;
    k[5] = (const void *)k_integrate_c32<STOP, kBlockC32Wide>;
}
static int variant_block(int variant) { return variant == kVariantC32Wide ? kBlockC32Wide : kBlock; }

template <bool STOP>
static void launch_variant(int variant, unsigned grid, hipStream_t st, const IntArgs &A)
{
    switch (variant) {
    case 0: hipLaunchKernelGGL((k_integrate<kPoleMonitor, GRAY_METRIC_KERR, STOP>), dim3(grid), dim3(kBlock), 0, st, A); break;
    case 1: hipLaunchKernelGGL((k_integrate_c32<STOP>), dim3(grid), dim3(kBlock), 0, st, A); break;
    case 2: hipLaunchKernelGGL((k_integrate<kPoleEulerCrossing, GRAY_METRIC_KERR, STOP>), dim3(grid), dim3(kBlock), 0, st, A); break;
    case 3: hipLaunchKernelGGL((k_integrate<kPoleNone, GRAY_METRIC_KERR, STOP>), dim3(grid), dim3(kBlock), 0, st, A); break;
    case kVariantC32Wide: hipLaunchKernelGGL((k_integrate_c32<STOP, kBlockC32Wide>), dim3(grid), dim3(kBlockC32Wide), 0, st, A); break;
    default: hipLaunchKernelGGL((k_integrate<kPoleMonitor, GRAY_METRIC_DEFORMED, STOP>), dim3(grid), dim3(kBlock), 0, st, A); break;
    }
}
static int variant_of(const gray_params *p, int metric)
{
    if (metric == GRAY_METRIC_DEFORMED) return 4;
    return p->precision == GRAY_FP32C ? 1 : (p->pole_mode == GRAY_POLE_MONITOR ? 0 : 1 + p->pole_mode);
}

struct DeviceInfo {
    int cus = 0;
    int blocks_per_cu[2][kVariants] = {};   // [honours the stop flag][variant]
};
static std::mutex g_dev_mutex;
static DeviceInfo g_dev[64];

static int device_info(DeviceInfo &out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error("hipGetDevice", e);
    if (dev < 0 || dev >= 64) return device_error("device index", hipErrorInvalidDevice);
    std::lock_guard<std::mutex> lk(g_dev_mutex);
    DeviceInfo &d = g_dev[dev];
    if (d.cus == 0) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return device_error("hipDeviceGetAttribute", e);
        const void *kernels[2][kVariants];
        variant_kernels<false>(kernels[0]);
        variant_kernels<true>(kernels[1]);
        for (int w = 0; w < 2; ++w)
            for (int v = 0; v < kVariants; ++v) {
                int nb = 0;
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernels[w][v], variant_block(v), 0);
                if (e != hipSuccess) return device_error("hipOccupancyMaxActiveBlocksPerMultiprocessor", e);
                d.blocks_per_cu[w][v] = nb > 0 ? nb : 1;
            }
        d.cus = cus;
    }
    out = d;
    return GRAY_OK;
}

// Workspace of gray_integrate_static, for callers that cannot allocate:
// one array per device, created with the code object and held until the
// process ends. Host code must never pass `scratch` itself to a kernel (on
// the host it names a stand-in, not device memory): static_scratch() looks
// up the device address once per device and every launch uses that.
static __device__ __align__(256) char scratch[GRAY_STATIC_WORKSPACE_BYTES];
static std::mutex g_scratch_mutex;
static void *g_scratch[64];

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
static int static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error("hipGetDevice", e);
    if (dev < 0 || dev >= 64) return device_error("device index", hipErrorInvalidDevice);
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_error("hipGetSymbolAddress(scratch)", e);
        if (!ptr || ((uintptr_t)ptr & 255u) != 0) return device_error("scratch address", hipErrorInvalidValue);
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return GRAY_OK;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

static size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Workspace: header, camera table, then (dense mode only) the ordering
// pass's per-block histograms, launch order and buckets. Offsets are
// multiples of 256 bytes.
struct WsLayout {
    size_t table, block_hist, perm, bucket, total;
};

static WsLayout ws_layout(int64_t n, int32_t ncam, uint32_t flags)
{
    WsLayout L{};
    L.table = kWsHeader;
    size_t off = L.table + round_up((size_t)ncam * sizeof(DevCam), 256);
    if (!(flags & GRAY_WORKLIST)) {
        L.block_hist = off;
        off += round_up((size_t)kOrderBlocks * kOrderBins * sizeof(unsigned), 256);
        L.perm = off;
        off += round_up((size_t)n * sizeof(int32_t), 256);
        L.bucket = off;
        off += round_up((size_t)n, 256);
    }
    L.total = off;
    return L;
}

} // namespace gray

using namespace gray;

extern "C" size_t gray_workspace_size(int64_t n, int32_t ncam, const gray_params *p)
{
    if (n < 0 || n > GRAY_MAX_PHOTONS || ncam < 1 || validate_params(p) != GRAY_OK) return 0;
    return ws_layout(n, ncam, p->flags).total;
}

static int launch_init(const gray_camera *cams, int32_t k0, int32_t cnt, const gray_params *p,
                       gray_state *s, hipStream_t st)
{
    InitArgs A;
    memset(&A, 0, sizeof A);
    A.x = s->x;
    A.lo = s->lo;
    A.status = s->status;
    A.steps = s->steps;
    A.cam = s->cam;
    A.counters = s->counters;
    A.mark = s->mark;
    A.disk = s->disk;
    if (p->flags & GRAY_WORKLIST) {
        A.work = s->work_in;
        A.work_count = s->work_in_count;
    }
    A.cam_done = s->cam_done;
    A.stride = s->stride;
    A.precision = p->precision;
    if (!fill_chunk(cams, k0, cnt, (p->flags & GRAY_SLOTS) != 0, A.ch)) return GRAY_OK;
    const int64_t m = A.ch.hi - A.ch.lo;
    hipLaunchKernelGGL(k_camera_init, dim3(blocks_for(m)), dim3(kBlock), 0, st, A);
    return check_launch("camera_init launch");
}

extern "C" int gray_camera_init(const gray_camera *cams, int32_t ncam, const gray_params *p, gray_state *s,
                                void *hip_stream)
{
    int e = validate_params(p);
    if (e) return e;
    if ((e = validate_state(s, p))) return e;
    if (s->n == 0) return GRAY_OK;
    if ((e = validate_cameras(cams, ncam, s->n, p->flags))) return e;
    int metric = 0;
    if ((e = call_metric(cams, ncam, p, &metric))) return e;
    hipStream_t st = (hipStream_t)hip_stream;
    for (int32_t k0 = 0; k0 < ncam; k0 += kCamChunk)
        if ((e = launch_init(cams, k0, ncam - k0 < kCamChunk ? ncam - k0 : kCamChunk, p, s, st))) return e;
    return GRAY_OK;
}

extern "C" int gray_camera_init_slot(const gray_camera *cams, int32_t ncam, int32_t slot, const gray_params *p,
                                     gray_state *s, void *hip_stream)
{
    int e = validate_params(p);
    if (e) return e;
    if (!(p->flags & GRAY_SLOTS)) return GRAY_EINVAL;
    if ((e = validate_state(s, p))) return e;
    if (s->n == 0) return GRAY_EINVAL;
    if ((e = validate_cameras(cams, ncam, s->n, p->flags))) return e;
    if (slot < 0 || slot >= ncam || (int64_t)cams[slot].nx * cams[slot].ny == 0) return GRAY_EINVAL;
    int metric = 0;
    if ((e = call_metric(cams, ncam, p, &metric))) return e;
    return launch_init(cams, slot, 1, p, s, (hipStream_t)hip_stream);
}

// Body of gray_integrate and gray_integrate_static once the arguments and
// the workspace have been checked: `workspace` is device memory of at least
// ws_layout(n, ncam, flags).total bytes, 256-byte aligned. Every byte the
// kernels read from it is written first by k_setup and the ordering passes
// of the same call, so its previous contents do not matter.
static int integrate_checked(const gray_camera *cams, int32_t ncam, const gray_params *p, gray_state *s, int metric,
                             void *workspace, const DeviceInfo &dev, hipStream_t st)
{
    int e = GRAY_OK;
    const bool wl = (p->flags & GRAY_WORKLIST) != 0;
    const WsLayout W = ws_layout(s->n, ncam, p->flags);
    char *ws = (char *)workspace;
    WsHeader *hdr = (WsHeader *)ws;
    DevCam *table = (DevCam *)(ws + W.table);

    for (int32_t k0 = 0; k0 < ncam; k0 += kCamChunk) {
        SetupChunk ch;
        memset(&ch, 0, sizeof ch);
        ch.base = k0;
        ch.count = ncam - k0 < kCamChunk ? ncam - k0 : kCamChunk;
        for (int j = 0; j < ch.count; ++j) {
            const gray_camera &c = cams[k0 + j];
            DevCam &d = ch.c[j];
            d.a = c.a;
            d.a2 = c.a * c.a;
            d.rbh = horizon_radius(c.a);
            d.rcap = d.rbh * (1.0 + p->horizon_eps);
            d.disk_rmin = p->disk_rmin < 0.0 ? isco_radius(c.a) : p->disk_rmin;
            d.disk_rmax = p->disk_rmax;
            d.eps3 = c.deform;
            d.call_steps = c.call_steps;
        }
        hipLaunchKernelGGL(k_setup, dim3(1), dim3(kWave), 0, st, table, hdr,
                           wl ? s->work_out_count : (unsigned *)nullptr, ch);
        if ((e = check_launch("setup launch"))) return e;
    }

    if (!wl) {
        // Launch order of the running photons (see k_order_key).
        OrderArgs O;
        memset(&O, 0, sizeof O);
        O.x = s->x;
        O.lo = s->lo;
        O.status = s->status;
        O.cam = s->cam;
        O.cams = table;
        O.bucket = (uint8_t *)(ws + W.bucket);
        O.block_hist = (unsigned *)(ws + W.block_hist);
        O.perm = (int32_t *)(ws + W.perm);
        O.hdr = hdr;
        O.n = s->n;
        O.stride = s->stride;
        O.precision = p->precision;
        const int64_t blocks = std::min<int64_t>(kOrderBlocks, blocks_for(s->n));
        O.per_block = (int64_t)round_up((size_t)((s->n + blocks - 1) / blocks), kBlock);
        const unsigned og = (unsigned)((s->n + O.per_block - 1) / O.per_block);
        hipLaunchKernelGGL(k_order_key, dim3(og), dim3(kBlock), 0, st, O);
        if ((e = check_launch("order key launch"))) return e;
        hipLaunchKernelGGL(k_order_scatter, dim3(og), dim3(kBlock), 0, st, O);
        if ((e = check_launch("order scatter launch"))) return e;
    }

    IntArgs A;
    memset(&A, 0, sizeof A);
    A.x = s->x;
    A.lo = s->lo;
    A.status = s->status;
    A.steps = s->steps;
    A.cam = s->cam;
    A.counters = s->counters;
    A.mark = s->mark;
    A.disk = s->disk;
    A.cams = table;
    A.queue = &hdr->queue;
    if (wl) {
        A.work_in = s->work_in;
        A.work_out = s->work_out;
        A.work_in_count = s->work_in_count;
        A.work_out_count = s->work_out_count;
    } else {
        A.work_in = (const int32_t *)(ws + W.perm);
        A.work_in_count = &hdr->count;
        A.two_ended = 1;
    }
    A.cam_done = s->cam_done;
    A.wave_iters = (unsigned long long *)s->wave_iters;
    A.stop = s->stop;
    A.n = s->n;
    A.stride = s->stride;
    A.step_frac = p->step_frac;
    A.xi_eps = p->xi_eps;
    A.euler_inv = 1.0 / p->euler_div;
    A.r_escape = p->r_escape;
    A.fp64_horizon = p->fp64_horizon;
    A.fp64_pole = p->fp64_pole;
    A.fp64_turn = p->fp64_turn;
    A.max_steps = p->max_steps;
    A.call_steps = p->call_steps;
    A.flags = p->flags;
    A.refill = 1;
    int variant = variant_of(p, metric);
    const bool stop = s->stop != nullptr;
    // FP32C: the FP64 wave of a block runs float photons while none waits
    // for it only when the launch is bound by throughput (work lists, or at
    // least kHelperPhotonsPerLane photons per float lane); a launch bound by
    // its longest photons keeps it free, so that a long photon that goes
    // over to FP64 is taken at once. A launch bound by throughput also takes
    // the wide block shape.
    const bool throughput = wl || s->n >= kHelperPhotonsPerLane * (int64_t)dev.cus * dev.blocks_per_cu[stop][variant] *
                                             (kBlock - kWave);
    A.helper = throughput;
    if (variant == 1 && throughput) variant = kVariantC32Wide;
    const int blk = variant_block(variant);
    const int64_t resident = (int64_t)dev.cus * dev.blocks_per_cu[stop][variant];
    // In work-list mode the list length is only known on the device; the grid
    // is capped at kMaxListWaves waves, which bounds the unused list tail.
    const int64_t need = wl ? std::min<int64_t>(resident, kMaxListWaves / (blk / kWave)) : (s->n + blk - 1) / blk;
    const unsigned grid = (unsigned)(need < resident ? need : resident);
    if (stop)
        launch_variant<true>(variant, grid, st, A);
    else
        launch_variant<false>(variant, grid, st, A);
    return check_launch("integrate launch");
}

static int validate_integrate(const gray_camera *cams, int32_t ncam, const gray_params *p, const gray_state *s,
                              int *metric)
{
    int e = validate_params(p);
    if (e) return e;
    if ((e = validate_state(s, p))) return e;
    if (s->n == 0) return GRAY_OK;
    if ((e = validate_cameras(cams, ncam, s->n, p->flags))) return e;
    if ((e = call_metric(cams, ncam, p, metric))) return e;
    // FP32C keeps its FP64-step count per photon: a photon that has taken
    // FP64 steps continues in FP64, also in a later call
    return p->precision == GRAY_FP32C && !s->counters ? GRAY_EINVAL : GRAY_OK;
}

extern "C" int gray_integrate(const gray_camera *cams, int32_t ncam, const gray_params *p, gray_state *s,
                              void *workspace, size_t workspace_bytes, void *hip_stream)
{
    int metric = 0;
    int e = validate_integrate(cams, ncam, p, s, &metric);
    if (e || s->n == 0) return e;
    if (!workspace || ((uintptr_t)workspace & 255u) != 0 ||
        workspace_bytes < gray_workspace_size(s->n, ncam, p))
        return GRAY_EWORKSPACE;
    DeviceInfo dev;
    if ((e = device_info(dev))) return e;
    return integrate_checked(cams, ncam, p, s, metric, workspace, dev, (hipStream_t)hip_stream);
}

extern "C" int gray_integrate_static(const gray_camera *cams, int32_t ncam, const gray_params *p, gray_state *s,
                                     void *hip_stream)
{
    int metric = 0;
    int e = validate_integrate(cams, ncam, p, s, &metric);
    if (e || s->n == 0) return e;
    const size_t need = gray_workspace_size(s->n, ncam, p);
    if (need == 0 || need > (size_t)GRAY_STATIC_WORKSPACE_BYTES) return GRAY_EWORKSPACE;
    DeviceInfo dev;
    if ((e = device_info(dev))) return e;
    void *ws = nullptr;
    if ((e = static_scratch(&ws))) return e;
    return integrate_checked(cams, ncam, p, s, metric, ws, dev, (hipStream_t)hip_stream);
}

extern "C" int gray_classify(const gray_camera *cams, int32_t ncam, const gray_params *p, const gray_state *s,
                             gray_result *out, void *hip_stream)
{
    int e = validate_params(p);
    if (e) return e;
    if ((e = validate_state(s, p))) return e;
    if (!out) return GRAY_EINVAL;
    if (s->n == 0) return GRAY_OK;
    if ((e = validate_cameras(cams, ncam, s->n, p->flags))) return e;
    int metric = 0;
    if ((e = call_metric(cams, ncam, p, &metric))) return e;
    if (!out->flag) return GRAY_EINVAL;
    const bool wl = (p->flags & GRAY_WORKLIST) != 0;
    if (wl && (out->xf || out->cons)) return GRAY_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    if (out->counts) {
        const int64_t m = (int64_t)ncam * 5;
        hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(m)), dim3(kBlock), 0, st, out->counts, m);
        if ((e = check_launch("classify zero launch"))) return e;
    }
    if (wl) {
        DeviceInfo dev;
        if ((e = device_info(dev))) return e;
        const int64_t grid = std::min<int64_t>((int64_t)dev.cus * 4, blocks_for(s->n));
        hipLaunchKernelGGL(k_classify_list, dim3((unsigned)grid), dim3(kBlock), 0, st, s->work_in,
                           s->work_in_count, s->status, s->cam, out->flag, out->counts, ncam);
        return check_launch("classify list launch");
    }
    for (int32_t k0 = 0; k0 < ncam; k0 += kCamChunk) {
        ClassArgs A;
        memset(&A, 0, sizeof A);
        A.x = s->x;
        A.lo = s->lo;
        A.status = s->status;
        A.mark = s->mark;
        A.flag = out->flag;
        A.xf = out->xf;
        A.cons = out->cons;
        A.counts = out->counts;
        A.stride = s->stride;
        A.precision = p->precision;
        if (!fill_chunk(cams, k0, ncam - k0 < kCamChunk ? ncam - k0 : kCamChunk,
                        (p->flags & GRAY_SLOTS) != 0, A.ch))
            continue;
        const int64_t cnt = A.ch.hi - A.ch.lo;
        hipLaunchKernelGGL(k_classify, dim3(blocks_for(cnt)), dim3(kBlock), 0, st, A);
        if ((e = check_launch("classify launch"))) return e;
    }
    return GRAY_OK;
}

extern "C" const char *gray_strerror(int code)
{
    switch (code) {
    case GRAY_OK: return "success";
    case GRAY_EINVAL: return "invalid argument";
    case GRAY_EDEVICE: return g_last_error;
    case GRAY_EWORKSPACE: return "workspace missing, misaligned or too small";
    case GRAY_EUNSUPPORTED: return "unsupported request";
    default: return "unknown error code";
    }
}

extern "C" int gray_version(void) { return 200; }

extern "C" size_t gray_struct_size(int which)
{
    switch (which) {
    case 0: return sizeof(gray_camera);
    case 1: return sizeof(gray_params);
    case 2: return sizeof(gray_state);
    case 3: return sizeof(gray_result);
    default: return 0;
    }
}
