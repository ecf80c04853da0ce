/*
 * libgbs: Gaussian beam summation on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the beam-summation stage of Gaussian beam tracing
 * (paper Sec. 2, Eq. (3)): given a traced ray table and observers, it sums
 * every nearby Gaussian beam (Eq. (1), with the dynamic-ray solution of
 * Eq. (2)) into each observer's complex pressure, and reports transmission
 * loss.  Inputs and outputs follow the paper's problem statement (Sec. 3.1
 * and Sec. 4.2: source, traced environment and observation points in,
 * pressure at the observation points out).
 *
 * Beam model.  For receiver R and segment j (start a, unit axis t, arc
 * length s0 at a, beam interval [lo, hi) along sigma = (R - a).t):
 *   n^2 = |R - a|^2 - sigma^2,  s = s0 + sigma,  q = s - i eps,  k = 2 pi f / c
 *   u   = (i k w / (8 pi^2)) prod(Gamma) (-i eps / q) exp(i k s + (i k / 2) n^2 / q)
 * kept iff lo <= sigma < hi and the Gaussian factor exp(-(k eps/2) n^2/|q|^2)
 * is >= exp(-gate_G).  P(R) = sum over the kept pairs, TL = -20 log10 |P|.
 * With atmospheric absorption (params.alpha) u also carries exp(-alpha s).
 * With anisotropic beams (params.eps_e2) Q = diag(q1, q2) (Eq. (1) with a
 * 2x2 Q; Eq. (2) with P = I/c): see gbs_params.eps_e2.
 * w is the launch solid angle of the segment's ray; prod(Gamma) the product of
 * the complex reflection coefficients of the faces the ray hit before the
 * segment.  A dense fan reproduces the unit monopole exp(ikr)/(4 pi r).
 *
 * Jobs.  A job is a (source, band) pair, job = src * n_freq + band; every job
 * has its own beam parameter eps[job].  All jobs run in one persistent launch.
 *
 * Memory.  Unless a flag says otherwise every pointer is DEVICE memory on the
 * context's device.  With GBS_FLAG_TABLE_HOST the ray and segment arrays are
 * host memory and are streamed to the device in chunks of at most
 * params.chunk_segs segments.  The caller owns every input and output; inputs
 * are read-only, outputs are caller-allocated and fully overwritten.  The
 * library never frees caller memory and keeps no caller pointer after a call
 * returns, except for graphs (gbs_graph_*), which hold the pointers given at
 * creation until gbs_graph_destroy.
 * Device scratch is held by the context and grows to what its calls need; it
 * includes the cull's batch records (up to 8 bands), sized from the largest
 * need seen and capped by the environment variable GBS_CULL_RECORD_BYTES
 * (bytes, read at each call; default 8 GiB, 0 turns the records off).  The
 * cap changes speed only: waves whose records do not fit are recomputed and
 * the results are the same bit for bit.
 *
 * Errors.  Every entry point returns GBS_OK (0) or a negative gbs_status;
 * gbs_last_error() describes the last failure on the context.  Sizes,
 * pointers and scalar parameters are checked on the host before any device
 * work.  Array contents are always checked (GBS_E_INVALID) before any beam is
 * evaluated: the ray CSR (ray_ptr[0] = 0, non-decreasing, ray_ptr[n_rays] =
 * n_segs; ray_src in [0, n_src) and non-decreasing), the face CSR
 * (face_ptr[0] = 0, non-decreasing; ids in [0, n_faces); n_faces > 0 when any
 * history is non-empty), finite a, s0, lo, hi with lo <= hi and |t| = 1
 * (+-1e-9), finite non-negative ray weights, finite receivers, frequencies,
 * beam parameters and absorption; in gbs_backward also finite lambda.  The
 * kernels that read these arrays flag problems in a device status word that
 * the host reads at its next synchronisation, so a failed call may already
 * have written zeros to its outputs; no kernel reads outside an array
 * because of bad contents.  No C++ exception crosses this interface.  Calls
 * on one context are not thread-safe; use one context per host thread.  Work
 * is enqueued on the context's stream; outputs are complete when that stream
 * is synchronised.  (A forward in several passes also runs its pair kernels
 * on two streams of its own, default priority; the context's stream waits
 * for each before it adds that pass into P, so the rule holds.)
 */
#ifndef GBS_H
#define GBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GBS_VERSION 4

typedef enum gbs_status {
    GBS_OK = 0,
    GBS_E_INVALID = -1,      /* bad argument (null, size, non-finite, range)     */
    GBS_E_OOM = -2,          /* device or host allocation failed                */
    GBS_E_HIP = -3,          /* a HIP runtime call failed (message has details) */
    GBS_E_UNSUPPORTED = -4,  /* valid request the library does not support      */
    GBS_E_STATE = -5         /* context/graph used in the wrong state           */
} gbs_status;

/* Arithmetic of the pair evaluation.
 * F64: everything in FP64.
 * MIX: geometry, arc length, normal distance and the phase in cycles with its
 *      reduction modulo one in FP64; Gaussian weight, sine/cosine, amplitude
 *      and complex products in FP32; per-receiver sums in FP64.
 * F32: everything in FP32 (ablation). */
typedef enum gbs_mode { GBS_MODE_F64 = 0, GBS_MODE_MIX = 1, GBS_MODE_F32 = 2 } gbs_mode;

/* params.flags */
#define GBS_FLAG_TABLE_HOST   1   /* ray/segment arrays are host memory: stream them */
#define GBS_FLAG_VALIDATE     2   /* accepted and ignored: contents are always checked */
#define GBS_FLAG_COUNT_ACTIVE 4   /* count kept pairs into gbs_stats (slower)          */
#define GBS_FLAG_TIME_KERNELS 8   /* time the pair kernel with HIP events (syncs)      */

typedef struct gbs_ctx gbs_ctx;

/* Rays: CSR over segments; rays sorted by source (ray_src non-decreasing). */
typedef struct gbs_rays {
    int32_t n_src;
    int64_t n_rays;
    const int64_t* ray_ptr;   /* [n_rays + 1], ray_ptr[0] = 0, last = n_segs   */
    const double* ray_w;      /* [n_rays] launch solid angle of each ray (sr)  */
    const int32_t* ray_src;   /* [n_rays] source index in [0, n_src)           */
} gbs_rays;

/* Segments: straight beam axes in table order (segments of ray i are
 * ray_ptr[i] .. ray_ptr[i+1]-1). */
typedef struct gbs_segs {
    int64_t n_segs;
    const double* a;          /* [n_segs * 3] start point (m)                  */
    const double* t;          /* [n_segs * 3] unit axis direction              */
    const double* s0;         /* [n_segs] arc length from the source at a (m)  */
    const double* lo;         /* [n_segs] beam interval start in sigma (m)     */
    const double* hi;         /* [n_segs] beam interval end, exclusive (m)     */
    const int64_t* face_ptr;  /* [n_segs + 1] CSR into face_ids                */
    const int32_t* face_ids;  /* faces hit before the segment, in hit order    */
    const double* e1;         /* [n_segs * 3] ray frame of anisotropic beams:
                                 a unit vector normal to t (+-1e-9), the axis of
                                 eps (params.eps_e2: e2 = t x e1 is the axis of
                                 eps_e2), carried along each ray and mirrored at
                                 every reflection; or NULL for e1 = z x t/|z x t|
                                 (x when t is vertical), the frame that the
                                 ground, roofs and walls of axis-aligned box
                                 scenes transport.  Only read with eps_e2.     */
} gbs_segs;

/* Faces: complex reflection coefficients (always device memory). */
typedef struct gbs_faces {
    int32_t n_faces;
    const double* gamma;      /* [n_faces * 2] (re, im)                         */
} gbs_faces;

typedef struct gbs_params {
    double c;                 /* speed of sound (m/s), > 0                       */
    double gate_G;            /* Gaussian gate exponent, > 0 (9.21 ~ 1e-4)       */
    int32_t mode;             /* gbs_mode                                        */
    int32_t flags;            /* GBS_FLAG_*                                      */
    int64_t chunk_segs;       /* max segments per pass; 0 = whole table          */
    int32_t rcv_per_lane;     /* pair kernel receivers per lane: 0 auto, 1, 2, 4 */
    int32_t work_chunk;       /* segments per pair-kernel work unit: 0 auto, else
                                 a power of two in [256, 65536]                 */
    const double* alpha;      /* [n_src * n_freq] atmospheric absorption per job
                                 (Np/m, finite, >= 0; device memory), or NULL
                                 for none: each beam's amplitude carries
                                 exp(-alpha s) along its arc length s.  The gate
                                 stays on the Gaussian factor alone.           */
    const double* eps_e2;     /* [n_src * n_freq] beam parameter along e2 per job
                                 (m, finite, > 0; device memory), or NULL for
                                 isotropic beams.  Anisotropic beams (Eq. (1)
                                 with Q = diag(q1, q2), q_m = s - i eps_m; eps
                                 of the call is eps_1): in the segment's ray
                                 frame (segs.e1, e2 = t x e1; a real symmetric
                                 initial width matrix is diagonal in the frame
                                 of its principal axes), with n1 = (R - a).e1
                                 and n2^2 = n^2 - n1^2,
                                   u = (i k w / (8 pi^2)) prod(Gamma)
                                       sqrt(q01/q1) sqrt(q02/q2) exp(i k s
                                       + (i k / 2)(n1^2/q1 + n2^2/q2))
                                 (principal roots: continuous along the beam),
                                 kept iff the Gaussian factor is >= exp(-gate_G).
                                 Every mode of gbs_forward and graphs; F64 and
                                 MIX in gbs_backward (which then also returns
                                 d_eps_e2); not with gbs_impulse_response
                                 (GBS_E_UNSUPPORTED).                          */
} gbs_params;

/* Plan statistics of the last forward/backward call on a context. */
typedef struct gbs_stats {
    int64_t dense_pairs;      /* sum over jobs of segments x receivers           */
    int64_t listed_pairs;     /* (segment, receiver) pairs left after culling    */
    int64_t active_pairs;     /* pairs kept by the gate (GBS_FLAG_COUNT_ACTIVE)  */
    int64_t n_items;          /* work items of the persistent pair kernel        */
    int32_t n_chunks;         /* passes over the table                           */
    int32_t patch_rcv;        /* receivers per work item                         */
    double ms_pairs;          /* pair-kernel time (the adjoint kernel's in gbs_backward),
                                 all passes (GBS_FLAG_TIME_KERNELS)                    */
    double ms_cull;           /* culling/list-building time (GBS_FLAG_TIME_KERNELS)   */
    int32_t grid;             /* workgroups of the last persistent launch          */
    int32_t blocks_per_cu;    /* resident workgroups per CU for that kernel        */
    int64_t scratch_bytes;    /* device scratch held by the forward's workspace;
                                 for gbs_forward_noalloc, the bytes of the static
                                 scratch that the call used                        */
} gbs_stats;

/* Create a context on `device` (HIP ordinal) that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context. */
int gbs_create(gbs_ctx** out, int device, void* hip_stream);

/* Release library-owned device scratch.  Safe on NULL. */
void gbs_destroy(gbs_ctx* ctx);

/* Change the stream later calls enqueue on. */
int gbs_set_stream(gbs_ctx* ctx, void* hip_stream);

/*
 * Forward beam summation (Eq. (3) discretised over the rays).
 *   rcv   [n_rcv * 3]            receiver positions (m)
 *   freqs [n_freq]               band frequencies (Hz), > 0
 *   eps   [n_src * n_freq]       beam parameter per job (m), > 0
 *   P     [n_src*n_freq*n_rcv*2] out: complex pressure (re, im), job-major
 *   TL    [n_src*n_freq*n_rcv]   out: -20 log10 |P| (+inf where P = 0); may be NULL
 * Deterministic: repeated calls with equal inputs give bitwise-equal P.
 */
int gbs_forward(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                const double* rcv, int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps,
                const gbs_params* params, double* P, double* TL);

/*
 * gbs_forward without any device allocation, for callers that cannot
 * allocate (code between HIP calls that must not allocate, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, outputs and
 * determinism as gbs_forward (bitwise the same P and TL); no hipMalloc,
 * hipFree or allocating library routine is called.  Every intermediate
 * buffer (receiver order, segment records, culled lists, work units,
 * partial sums) is carved from one static device array of 128 MiB per GPU,
 * loaded with the library's code object and held until the process ends;
 * its device address is looked up once per device by gbs_create.
 * Limits and errors:
 *   - a call whose buffers need more than 128 MiB returns GBS_E_UNSUPPORTED
 *     (message names the buffer); the check runs as the plan is laid out,
 *     so P may already be zeroed and TL is untouched.  The 2,000-ray open
 *     plane over 64 x 64 receivers needs a few MiB; gbs_stats.scratch_bytes
 *     reports what a call used;
 *   - device tables only: GBS_FLAG_TABLE_HOST returns GBS_E_UNSUPPORTED;
 *   - the array is shared by every call on a GPU, from every context and
 *     stream, and keeps the last call's contents (each call clears what must
 *     start at zero).  Calls that overlap on one GPU race: issue them on one
 *     stream, or wait for one call's work before starting the next.
 * Like gbs_forward it synchronises the stream once to size the culled lists.
 */
int gbs_forward_noalloc(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                        const double* rcv, int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps,
                        const gbs_params* params, double* P, double* TL);

/*
 * Adjoint of gbs_forward for dL = Re sum_{job,r} lambda[job,r] * dP[job,r],
 * with the ray geometry and the gate's active set held fixed (F64 and MIX).
 *   lambda  [n_src*n_freq*n_rcv*2]  (re, im)
 *   d_gamma [n_faces * 2]  out: (dL/dRe Gamma_f, dL/dIm Gamma_f)
 *   d_rcv   [n_rcv * 3]    out: dL/dR
 *   d_eps   [n_src*n_freq] out: dL/deps per job (anisotropic beams: dL/deps_1)
 *   d_eps_e2 [n_src*n_freq] out: dL/deps_e2 per job with anisotropic beams
 *                          (params.eps_e2; ignored without), with the frame
 *                          held fixed:
 *     d ln u/dR = t (ik - (1/q1 + 1/q2)/2 - (ik/2)(n1^2/q1^2 + n2^2/q2^2) - alpha)
 *                 + (ik n1/q1) e1 + (ik n2/q2) e2,
 *     d ln u/deps_m = (1/eps_m + i/q_m)/2 - (k/2) n_m^2/q_m^2
 * Any output pointer may be NULL to skip it.  Deterministic: repeated calls
 * with equal inputs give bitwise-equal outputs (receiver and beam-parameter
 * sums are reduced in a fixed order; the per-segment and per-face sums
 * behind d_gamma are exact fixed-point sums with a resolution of 2^-92 of a
 * bound on them, whose value does not depend on the order of accumulation).
 */
int gbs_backward(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                 const double* rcv, int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps,
                 const gbs_params* params, const double* lambda, double* d_gamma, double* d_rcv,
                 double* d_eps, double* d_eps_e2);

/* Statistics of the last gbs_forward / gbs_backward on ctx. */
int gbs_get_stats(const gbs_ctx* ctx, gbs_stats* out);

/*
 * Graphs (batched replay; an extension, not in the paper): capture one forward call (all
 * jobs, one persistent launch per pass over the table) into a hipGraph and
 * replay it.  Creation runs the full plan once (receiver ordering, culling,
 * work lists for every pass) and captures the per-call work: for each pass
 * the table slice (copied from host memory with GBS_FLAG_TABLE_HOST, which
 * then must be page-locked), the segment records and the pair kernel.
 * Between replays the caller may change the CONTENTS of faces->gamma and of a
 * host table's arrays, but not the geometry, receivers, frequencies, eps,
 * params.eps_e2 or params.alpha (the culled work lists and the per-job
 * constants are baked in).  The graph holds the pointers given
 * at creation.
 */
typedef struct gbs_graph gbs_graph;
int gbs_graph_create(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                     const double* rcv, int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps,
                     const gbs_params* params, double* P, double* TL, gbs_graph** out);
int gbs_graph_launch(gbs_graph* g);
void gbs_graph_destroy(gbs_graph* g);

/*
 * Autotuner (an extension; the paper has none): times the forward on
 * the given problem for every candidate pair-kernel shape (receivers per
 * lane 1, 2, 4) and work-unit size (1024, 2048, 4096 segments) and stores the
 * fastest in the context for `params.mode`; later calls with rcv_per_lane or
 * work_chunk 0 use it.  Writes the choice to *rcv_per_lane and *work_chunk
 * when non-NULL.  P [n_src*n_freq*n_rcv*2] is scratch output.
 */
int gbs_autotune(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                 const double* rcv, int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps,
                 const gbs_params* params, double* P, int32_t* rcv_per_lane, int32_t* work_chunk);

/*
 * Broadband synthesis (the time-domain form of Eq. (1); the paper steps its
 * field in time, Table 2): the forward sum at the n_bins frequencies
 * f_n = (bin0 + n) df, windowed and transformed to a real time signal per
 * (source, receiver).  With the exp(-i omega t) convention,
 *   h[src][r][m] = 2 df Re sum_n w_n P_n(src, r) exp(-2 pi i f_n m dt),
 *   dt = 1 / (n_fft df),  m < n_t,
 * a length-n_fft transform of the zero-padded spectrum (period 1/df: choose
 * df below c / (longest path) to avoid wrap-around).
 *   eps    [n_src * n_bins]  beam parameter per (source, bin), > 0 (device)
 *   window [n_bins]          real taper w_n (device), or NULL for 1
 *   params                   as for gbs_forward; params.alpha, if set, is
 *                            [n_src * n_bins]
 *   h      [n_src * n_rcv * n_t] out (device)
 * n_fft a power of two in [64, 4096]; 1 <= bin0; bin0 + n_bins <= n_fft / 2;
 * 1 <= n_t <= n_fft.  Runs gbs_forward over chunks of at most 64 bins
 * (synchronising the stream between chunks), then one transform per row.
 * Scratch: n_src * n_rcv * n_fft complex doubles.
 */
int gbs_impulse_response(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                         const double* rcv, int64_t n_rcv, double df, int32_t bin0, int32_t n_bins,
                         const double* eps, const double* window, const gbs_params* params, int32_t n_fft,
                         int32_t n_t, double* h);

/*
 * Ray tracing: the stage before beam summation (Sec. 3.1; one thread per ray
 * as in Sec. 3.3).  Traces a fan of rays through a scene of the ground plane
 * z = 0 (face 0) and axis-aligned boxes standing on it, with specular
 * reflection (image-source geometry, Sec. 1), at most max_refl reflections
 * per ray (R_max of Tables 2 and 3), until each ray's arc length reaches
 * s_max, and writes the ray table that gbs_forward reads.
 *
 * Scene.  Box b occupies [x0, x1] x [y0, y1] x [0, h] and owns the faces
 * 1 + b*5*panels^2 ... : walls -x, +x, -y, +y, then the roof, each split into
 * panels x panels cells (cell = iu * panels + iv, u along the face's first
 * in-plane axis (y for x-walls, x otherwise), v along the second (z for
 * walls, y for the roof)).  n_faces of the table = 1 + n_boxes*5*panels^2.
 *
 * Rules.  Hits need a distance > 1e-7 m; a box's entry face is on the first
 * axis whose slab entry equals the entry distance; a box is never entered
 * through its floor; the ground wins a tie with a box, the lower box index
 * a tie between boxes.  Beam extents: walls and roofs truncate (lo = 0,
 * hi = L); the ground is transparent (a segment ending on it has
 * hi = L + L_next, the next segment lo = -L).  image_complete (no boxes):
 * a ray that never reflects from the ground gets a second segment from the
 * source mirrored in z = 0 along the mirrored direction, lo = 0, hi = s_max,
 * face history [0].  Segment j of a ray has the end faces of segments
 * 0..j-1 as its history.  All arithmetic is IEEE double without fused
 * multiply-adds: the table is deterministic and identical for any launch.
 */
typedef struct gbs_scene {
    int32_t n_boxes;          /* >= 0                                            */
    int32_t panels;           /* 1..8                                            */
    const double* boxes;      /* [n_boxes * 5] x0, x1, y0, y1, h (device);
                                 x0 < x1, y0 < y1, h > 0, finite                 */
    double s_max;             /* arc length at which every ray ends (m), > 0     */
    int32_t max_refl;         /* R_max, 0..32                                    */
    int32_t image_complete;   /* 0/1; 1 needs n_boxes == 0                       */
} gbs_scene;

/* Launch fan: rays from their sources (device memory). */
typedef struct gbs_fan {
    int32_t n_src;
    const double* src_xyz;    /* [n_src * 3], z > 0                              */
    int64_t n_rays;           /* >= 0                                            */
    const double* dirs;       /* [n_rays * 3] unit directions (|d|^2 = 1 +- 1e-9) */
    const int32_t* ray_src;   /* [n_rays] source of each ray in [0, n_src),
                                 non-decreasing, or NULL for source 0            */
    const double* s_max_src;  /* [n_src] arc-length budget per source (m, > 0;
                                 device), or NULL for scene.s_max everywhere     */
    const double* e1;         /* [n_rays * 3] launch frame of anisotropic beams
                                 (unit, normal to the direction +-1e-9; device),
                                 or NULL: gbs_trace then writes no frames       */
} gbs_fan;

/*
 * Sizes of the table gbs_trace will write: *n_segs segments and *n_face_ids
 * face-history entries.  Synchronises the context's stream.  *token (if
 * non-NULL) receives a nonzero token: passed to the next gbs_trace on this
 * context with the same arguments and unchanged input contents, it lets
 * gbs_trace reuse this count instead of tracing twice.
 */
int gbs_trace_count(gbs_ctx* ctx, const gbs_scene* scene, const gbs_fan* fan, int64_t* n_segs,
                    int64_t* n_face_ids, int64_t* token);

/*
 * Trace the fan and write the table (device memory, caller-allocated).
 * token: 0, or the token of the last gbs_trace_count on this context for the
 * same scene and fan (GBS_E_INVALID if it is not; any trace call in between
 * invalidates it); the caller guarantees the inputs did not change.
 *   ray_ptr  [n_rays + 1]    CSR of each ray's segments
 *   seg_a, seg_t [cap_segs * 3], seg_s0, seg_lo, seg_hi [cap_segs]
 *   face_ptr [cap_segs + 1]  CSR into face_ids
 *   face_ids [cap_face_ids]
 *   seg_e1   [cap_segs * 3]  optional (NULL to skip; needs fan.e1): the launch
 *                            frame carried to every segment, mirrored at each
 *                            reflection like the direction (the image segment
 *                            of the open plane: mirrored in z = 0), for
 *                            gbs_segs.e1
 * The ray weights and sources of the table are the caller's (unchanged).
 * *n_segs and *n_face_ids receive the sizes; a capacity below them is
 * GBS_E_INVALID (nothing written past the capacities).  A direction that is
 * not a unit vector is GBS_E_INVALID.  Synchronises the context's stream
 * once (to read the sizes) before the table is written.
 */
int gbs_trace(gbs_ctx* ctx, const gbs_scene* scene, const gbs_fan* fan, int64_t token, int64_t cap_segs,
              int64_t cap_face_ids, int64_t* ray_ptr, double* seg_a, double* seg_t, double* seg_s0,
              double* seg_lo, double* seg_hi, int64_t* face_ptr, int32_t* face_ids, double* seg_e1,
              int64_t* n_segs, int64_t* n_face_ids);

/*
 * Atmospheric attenuation of a pure tone in dB per metre: the model of
 * ISO 9613-1 (water-vapour concentration from the relative humidity, oxygen
 * and nitrogen relaxation frequencies, classical and rotational absorption)
 * for the atmosphere the paper's runs specify (Tables 2 and 3: temperature,
 * relative humidity, pressure; 20 deg C, 70 %, 1 atm there).  As an
 * amplitude decay rate for gbs_params.alpha: alpha = dB/m * ln(10) / 20.
 * Host function; needs no context or device.  NaN for arguments outside
 * f > 0, -100 < temp_c < 100, 0 <= rh_pct <= 100, pressure_atm > 0.
 */
double gbs_air_absorption_db(double f_hz, double temp_c, double rh_pct, double pressure_atm);

/* Message describing the last error on ctx (never NULL). */
const char* gbs_last_error(const gbs_ctx* ctx);

/* GBS_VERSION of the built library. */
int gbs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GBS_H */
