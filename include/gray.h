/*
 * gray.h -- C ABI of the MI355X (gfx950) Kerr photon-geodesic integrator.
 *
 * The library traces null geodesics of the Kerr spacetime backwards from an
 * image plane, one independent photon per GPU lane, with the scheme of
 * Chan, Psaltis & Ozel (2013), "GRay", Sec. 2: classical fourth-order
 * Runge-Kutta on the second-order geodesic equations in Boyer-Lindquist
 * coordinates (G = c = M = 1), the adaptive step of eq. (2), the horizon stop,
 * the theta remap of eq. (3) and the null-condition monitor of eq. (4) with
 * its forward-Euler re-integration at h/9.
 *
 * Conventions shared by every entry point
 *   - All functions are C linkage, never throw, and return a gray_err code.
 *   - Device buffers are allocated and freed by the caller; the library never
 *     allocates device or host memory. Camera and parameter structs are host
 *     memory and are consumed before the call returns (they travel as kernel
 *     arguments), so the caller may reuse them immediately.
 *   - Every call enqueues work on `hip_stream` (a hipStream_t; NULL = the
 *     null stream) and returns without synchronising. Calls on different
 *     streams with disjoint buffers and workspaces are independent. Two calls
 *     that share a workspace must be ordered by the caller.
 *   - Argument errors are detected on the host before anything is enqueued
 *     and return GRAY_EINVAL (nothing is touched). A failed launch returns
 *     GRAY_EDEVICE; gray_strerror() then describes it. Numerical failure is
 *     per photon (status GRAY_NONFINITE), never a call error.
 *   - n == 0 is valid and enqueues nothing.
 *   - Shape of the interface: gray_camera_init needs no workspace;
 *     gray_integrate takes its workspace with its size; every per-photon
 *     array, outputs included (counters, mark, disk record), lives in
 *     gray_state; a time-bounded integrate call is a step budget
 *     (gray_params.call_steps), and a running call can be stopped early
 *     through gray_state.stop.
 *
 * Photon state (gray_state), structure of arrays in device memory
 *   x      component-major, 8 rows of `stride` elements:
 *          row c holds component c of every photon, c = 0..7 for
 *          (t, r, theta, phi, k^t, k^r, k^theta, k^phi); element type is
 *          double for GRAY_FP64 and float (the high word) for GRAY_FP32C.
 *          k is the integrated tangent; the photon's physical momentum is
 *          p = -k (the ray is traced from the observer back to the hole).
 *   lo     GRAY_FP32C only: float compensation words, same shape as x; the
 *          state is hi + lo. Must be NULL for GRAY_FP64.
 *   status int32[n]  gray_status of each photon.
 *   steps  int32[n]  accepted steps taken so far.
 *   cam    int32[n]  camera index of each photon (written by camera_init).
 *   counters  int32, 3 rows of `stride`: Euler fallbacks (eq. 4),
 *          theta remaps (eq. 3), steps taken in FP64 (GRAY_FP32C; 0 else).
 *          Optional, except for gray_integrate in GRAY_FP32C.
 *   mark   optional double, 8 rows of `stride`: the last accepted state with
 *          r >= 2 r_bh before the photon last fell below 2 r_bh (drift
 *          diagnostics for captured photons; r = 0 if never marked).
 *   disk   optional double, 3 rows of `stride`: first equatorial crossing
 *          inside the recorder window (r_c, phi_c, redshift g); all zero
 *          when there was none. Required when GRAY_RECORD_DISK is set.
 *   stride must be >= n and a multiple of 64; all rows are stride apart.
 *   work_in, work_out, work_in_count, work_out_count
 *          work-list mode only (GRAY_WORKLIST), else NULL: int32 photon-id
 *          lists of capacity n + GRAY_WORKLIST_SLACK each, and their uint32
 *          lengths, all device memory. gray_integrate advances the photons listed in
 *          work_in[0 .. *work_in_count) and appends to work_out the ids that
 *          are still GRAY_RUNNING when it stops (it zeroes *work_out_count
 *          first; the order of ids is unspecified, and entries equal to -1 are
 *          unused space that readers skip). gray_camera_init_slot
 *          appends the new slot's ids to work_in. A caller that iterates swaps
 *          (work_in, work_in_count) with (work_out, work_out_count) between
 *          integrate calls, so each call's work is the live photons only.
 *          gray_classify in this mode classifies only the photons listed in
 *          work_in (flag and counts; xf and cons must be NULL).
 */
#ifndef GRAY_H
#define GRAY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GRAY_OK = 0,
    GRAY_EINVAL = -1,       /* bad argument; nothing was enqueued            */
    GRAY_EDEVICE = -2,      /* HIP runtime or launch failure                 */
    GRAY_EWORKSPACE = -3,   /* workspace NULL or smaller than required       */
    GRAY_EUNSUPPORTED = -4  /* valid request the library does not serve     */
} gray_err;

typedef enum {
    GRAY_FP64 = 0,  /* all arithmetic in double                               */
    GRAY_FP32C = 1  /* float steps on a compensated (hi + lo) state; a photon
                       continues in double precision once it enters a zone
                       named in gray_params (near the horizon, a pole, a
                       radial turning point) or once a float step cannot
                       decide the null monitor of eq. (4). Requires the
                       counters array (its FP64-step count marks those
                       photons, so a later call continues them in FP64).  */
} gray_precision;

typedef enum {
    GRAY_RUNNING = 0,    /* still integrating (resumable)                     */
    GRAY_CAPTURED = 1,   /* r < r_bh (1 + horizon_eps): horizon stop, Sec. 2  */
    GRAY_ESCAPED = 2,    /* r > r_escape while moving outward                 */
    GRAY_UNFINISHED = 3, /* max_steps reached                                 */
    GRAY_NONFINITE = 4   /* non-finite state or step size                     */
} gray_status;

/* gray_params.flags */
#define GRAY_RECORD_DISK 1u /* record the first equatorial crossing (Sec. 3) */
#define GRAY_WORKLIST 4u    /* work-list mode, see gray_state                */
#define GRAY_WORKLIST_SLACK (1 << 20) /* extra list entries a call may leave unused */
#define GRAY_MAX_PHOTONS 2147482623LL /* largest n (2^31 - 1025): photon ids, launch
                                         order and queue positions are 32-bit */
#define GRAY_SLOTS 2u       /* slot mode, for callers that keep many requests in
                               one resident photon pool (continuous batching):
                               `cams` is a slot table and camera k covers photon
                               ids [first, first + nx * ny) in any order; ranges
                               are disjoint and inside [0, n); nx * ny == 0
                               marks a free slot. The camera index stored per
                               photon is the slot index. Photons outside every
                               camera are ignored by camera_init and classify
                               and must not be GRAY_RUNNING for integrate.   */

/* gray_camera.kind */
typedef enum {
    GRAY_CAMERA_GRID = 0,  /* cell-centred Cartesian grid in (alpha, beta)        */
    GRAY_CAMERA_POLAR = 1  /* polar grid (R, vartheta) about the image centre, as
                              in the photon-ring study of Sec. 4                 */
} gray_camera_kind;

/* gray_camera.metric: the spacetime the camera looks at */
typedef enum {
    GRAY_METRIC_KERR = 0,     /* Kerr, spin a (deform must be 0)                    */
    GRAY_METRIC_DEFORMED = 1  /* Kerr deformed by the Johannsen-Psaltis deviation
                                 function h = deform * r / Sigma^2 (deform = their
                                 epsilon_3; deform = 0 is Kerr), a non-Kerr
                                 spacetime without a Carter constant, the case
                                 Sec. 1 gives for integrating the second-order
                                 equations:
                                   g_tt   = -(1 + h)(1 - 2 r / Sigma)
                                   g_tphi = -(2 a r sin^2 / Sigma)(1 + h)
                                   g_rr   = Sigma (1 + h) / (Delta + a^2 sin^2 h)
                                   g_thth = Sigma
                                   g_phph = sin^2 (r^2 + a^2 + 2 a^2 r sin^2 / Sigma)
                                            + h a^2 (Sigma + 2 r) sin^4 / Sigma
                                 Requires deform >= 0 (or a = 0 and deform > -8),
                                 where the metric is regular outside the Kerr
                                 horizon r_bh, which the step-size rule and the
                                 capture radius keep using. Served in GRAY_FP64
                                 with GRAY_POLE_MONITOR and without
                                 GRAY_RECORD_DISK (GRAY_EUNSUPPORTED otherwise);
                                 all cameras of a call share one metric kind.
                                 gray_classify reports E and L_z in this metric
                                 (constants of motion) and Carter's Q in its Kerr
                                 form, which drifts when deform != 0.          */
} gray_metric;

/* One camera: a Kerr hole of spin a seen from distance r_obs at inclination
 * incl (radians from the spin axis, azimuth 0), with a regular nx * ny grid
 * on a flat image plane perpendicular to the line of sight (Sec. 2 and Sec. 3
 * place the image plane at r = 1000 M). Pixel (ix, iy) is photon
 * first + iy * nx + ix and has image-plane coordinates (alpha along +phi,
 * beta towards the spin axis)
 *   GRAY_CAMERA_GRID:
 *     alpha = alpha_lo + (alpha_hi - alpha_lo) (ix + 1/2) / nx
 *     beta  = beta_lo  + (beta_hi  - beta_lo)  (iy + 1/2) / ny
 *   GRAY_CAMERA_POLAR (alpha_* bound the radius R, beta_* the angle):
 *     R = alpha_lo + (alpha_hi - alpha_lo) (ix + 1/2) / nx
 *     vartheta = beta_lo + (beta_hi - beta_lo) iy / (ny - 1)  (beta_lo if ny = 1)
 *     alpha = R cos(vartheta),  beta = R sin(vartheta)
 * Constraints: 0 <= a < 1, r_obs > r_bh = 1 + sqrt(1 - a^2), 0 <= incl <= pi,
 * nx, ny >= 1, finite ranges, kind one of gray_camera_kind. Cameras passed
 * together must tile [0, n) in order with no gaps (unless GRAY_SLOTS is
 * set). */
typedef struct {
    double a, r_obs, incl;
    int32_t nx, ny;
    double alpha_lo, alpha_hi, beta_lo, beta_hi;
    int64_t first;
    int32_t kind;      /* gray_camera_kind */
    int32_t metric;    /* gray_metric      */
    double deform;     /* deviation of GRAY_METRIC_DEFORMED; 0 for Kerr */
    int32_t call_steps; /* >= 0; used by gray_integrate only when
                           gray_params.call_steps > 0: if > 0, this camera's
                           photons advance at most this many steps in the
                           call instead of gray_params.call_steps (a serving
                           loop gives a request whose last photons are
                           running a larger budget); 0: gray_params'.     */
    int32_t reserved;  /* 0 */
} gray_camera;

/* Treatment of steps near the polar axis, where Boyer-Lindquist coordinates
 * are singular (Sec. 2, Fig. 2). The production scheme is the default; the
 * other two are the paper's earlier treatments, kept for comparison. */
typedef enum {
    GRAY_POLE_MONITOR = 0,        /* production: when the RK4 step violates the
                                     null condition eq. (4) by more than xi_eps,
                                     re-integrate it with one forward-Euler step
                                     of h / euler_div                          */
    GRAY_POLE_EULER_CROSSING = 1, /* when the RK4 step ends across a pole
                                     (theta outside [0, pi]), replace it by one
                                     forward-Euler step of the same h          */
    GRAY_POLE_NONE = 2            /* RK4 and the remap of eq. (3) only          */
} gray_pole_mode;

/* Integrator parameters (Sec. 2 names them Delta, delta and epsilon). */
typedef struct {
    double step_frac;    /* Delta of the step-size rule eq. (2); ~1/32      > 0 */
    double horizon_eps;  /* capture when r < r_bh (1 + horizon_eps)          > 0 */
    double r_escape;     /* escape when r > r_escape and k^r > 0             > 0 */
    double xi_eps;       /* epsilon of eq. (4); ~1e-3                        > 0 */
    double euler_div;    /* Euler fallback step h / euler_div; 9 in Sec. 2  >= 1 */
    double disk_rmin;    /* recorder window [rmin, rmax]; rmin < 0: r_ISCO(a)     */
    double disk_rmax;
    /* GRAY_FP32C only: a photon continues in double precision from the
     * first step at which any of these holds (near the horizon, near a pole,
     * near a radial turning point); all >= 0, 0 disables a zone; e.g.
     * 0.02, 0, 0 (float rounding near the horizon is amplified by 1/Delta;
     * the float step keeps its digits next to the poles without a zone).    */
    double fp64_horizon; /* r < r_bh (1 + fp64_horizon)                          */
    double fp64_pole;    /* sin(theta) < fp64_pole                                */
    double fp64_turn;    /* |k^r| < fp64_turn |k^t|                               */
    int32_t max_steps;   /* total accepted steps before GRAY_UNFINISHED     >= 1 */
    int32_t call_steps;  /* > 0: advance each photon at most this many steps in
                            this call and leave it GRAY_RUNNING (resumable);
                            0: run to termination                                */
    int32_t precision;   /* gray_precision                                       */
    uint32_t flags;      /* GRAY_RECORD_DISK                                     */
    int32_t pole_mode;   /* gray_pole_mode; GRAY_FP32C supports GRAY_POLE_MONITOR
                            only (GRAY_EUNSUPPORTED otherwise)                  */
    int32_t reserved;    /* 0                                                    */
} gray_params;

typedef struct {
    void *x;
    void *lo;
    int32_t *status;
    int32_t *steps;
    int32_t *cam;
    int32_t *counters;
    double *mark;
    double *disk;
    int64_t n;
    int64_t stride;
    int32_t *work_in;
    int32_t *work_out;
    uint32_t *work_in_count;
    uint32_t *work_out_count;
    uint32_t *cam_done;   /* optional [ncam]: photons of each camera that have
                             stopped in a terminal status; camera_init (and
                             camera_init_slot for its slot) zeroes the entry,
                             gray_integrate adds to it as photons stop       */
    uint64_t *wave_iters; /* optional [1]: gray_integrate adds the number of
                             loop iterations its waves ran with at least one
                             photon (each advances every busy lane by one
                             step); the caller zeroes it. Lane efficiency of
                             a call = photon-steps / (64 * wave_iters)       */
    const uint32_t *stop; /* optional [1]: a stop request to a running
                             gray_integrate (a watchdog), in device memory or
                             in host memory mapped for the device (the
                             library reads it past the caches and never
                             writes it). Each wave reads it every 64 of its
                             loop iterations; once it reads non-zero, every
                             photon the wave holds or takes from then on is
                             stored after its next step, as at the end of
                             call_steps (GRAY_RUNNING unless that step ended
                             it; in work-list mode it goes on to work_out),
                             so the call ends after about one step per
                             remaining photon. In GRAY_FP32C a photon that
                             needs an FP64 step is stored without taking it,
                             and the photons of a block's FP64 wave are
                             stored after their next step once the block's
                             float waves have exited. A later call
                             continues every photon bit for bit.           */
} gray_state;

/* Outputs of gray_classify, all device memory, all rows `stride` apart
 * (the state's stride). */
typedef struct {
    int8_t *flag;     /* required [n]: gray_status of each photon              */
    double *xf;       /* optional 8 rows: final state in double (FP32C: hi+lo) */
    double *cons;     /* optional 9 rows: E0, L0, Q0 at the camera; E, L, Q at the
                         final state; drifts dE = |E/E0 - 1|,
                         dL = |L - L0| / (|L0| + E0),
                         dQ = |Q - Q0| / (|Q0| + L0^2 + E0^2), evaluated at the
                         final state, or for captured photons at `mark` when the
                         state carries one                                     */
    int32_t *counts;  /* optional [ncam][5]: photons per camera and status     */
} gray_result;

/* Bytes of device workspace that gray_integrate needs for n photons over ncam
 * cameras: per-camera constants and the queue counter, plus, without
 * GRAY_WORKLIST, the launch order (5 bytes per photon and a fixed 256 KiB of
 * histograms). Returns 0 on invalid arguments. */
size_t gray_workspace_size(int64_t n, int32_t ncam, const gray_params *p);

/* Image plane -> initial state (Sec. 2 defers the set-up; see the camera
 * comment). Writes x (and lo), status = GRAY_RUNNING, steps = 0, cam, and
 * clears counters, mark and disk when present. */
int gray_camera_init(const gray_camera *cams, int32_t ncam, const gray_params *p,
                     gray_state *s, void *hip_stream);

/* Slot mode (GRAY_SLOTS must be set in p->flags): initialise only the photons
 * of cams[slot] (ids [first, first + nx * ny)), storing `slot` as their camera
 * index; the rest of the state is untouched. Same layout and ownership rules
 * as gray_camera_init. Returns GRAY_EINVAL when slot is outside [0, ncam), the
 * slot is empty, or the slot table is invalid. */
int gray_camera_init_slot(const gray_camera *cams, int32_t ncam, int32_t slot,
                          const gray_params *p, gray_state *s, void *hip_stream);

/* Integrate every GRAY_RUNNING photon with the scheme of Sec. 2 until it is
 * captured, escapes, turns non-finite or reaches max_steps (or until it has
 * taken call_steps steps in this call). Photons of all cameras share one
 * persistent launch; a wave refills lanes whose photon finished from a global
 * queue. Without GRAY_WORKLIST the queue holds the running photons ordered
 * so that those expected to take the most steps (constants of motion near a
 * spherical photon orbit, or small |L_z|: paths near the polar axis) start
 * first; the order never changes a photon's result. Resumable: the state is
 * the checkpoint, and repeated calls with call_steps > 0 reproduce a single
 * call bit for bit (in GRAY_FP32C too: its FP64 steps round the state to
 * the float pair it is stored as). A time-bounded call is expressed as this
 * step budget rather than a time limit, so that where a photon pauses never
 * depends on timing.
 * workspace: device memory of gray_workspace_size() bytes, 256-byte aligned. */
int gray_integrate(const gray_camera *cams, int32_t ncam, const gray_params *p,
                   gray_state *s, void *workspace, size_t workspace_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * integration as gray_integrate, with the workspace taken from a static
 * device array of GRAY_STATIC_WORKSPACE_BYTES that the library holds on each
 * device it runs on until the process ends. The call allocates nothing; the
 * caller still owns every buffer of `s`. Returns GRAY_EWORKSPACE when
 * gray_workspace_size(s->n, ncam, p) exceeds GRAY_STATIC_WORKSPACE_BYTES
 * (without GRAY_WORKLIST that is about 6.6M photons; with it, the camera
 * table alone). Every call on one device shares that device's array, and
 * the array keeps the last call's contents (each call rewrites what it
 * reads): calls that overlap on one device, on different streams or from
 * different threads, race and must be ordered by the caller. */
#define GRAY_STATIC_WORKSPACE_BYTES (32u << 20)
int gray_integrate_static(const gray_camera *cams, int32_t ncam, const gray_params *p,
                          gray_state *s, void *hip_stream);

/* Final classification and conservation diagnostics (E, L_z and Carter's Q,
 * Sec. 1) of every photon; see gray_result. */
int gray_classify(const gray_camera *cams, int32_t ncam, const gray_params *p,
                  const gray_state *s, gray_result *out, void *hip_stream);

/* Static description of an error code; for GRAY_EDEVICE, of the last device
 * error seen by the calling thread. Never NULL. */
const char *gray_strerror(int code);

/* Library version as an integer MAJOR * 10000 + MINOR * 100 + PATCH. */
int gray_version(void);

/* sizeof of the ABI structs, for bindings to check their mirrors:
 * which = 0 gray_camera, 1 gray_params, 2 gray_state, 3 gray_result;
 * 0 for any other value. */
size_t gray_struct_size(int which);

#ifdef __cplusplus
}
#endif
#endif /* GRAY_H */
