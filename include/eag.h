/*
 * eag.h - C ABI of the MI355X (gfx950) surfel ray/path tracing library.
 *
 * Scope: ray tracing through a scene of 2D Gaussian surfels as defined in
 * "EAG-PT: Emission-Aware Gaussians and Path Tracing for Diffuse Indoor
 * Scene Reconstruction and Editing" (arXiv 2601.23065):
 *   - the surfel and its response              Sec. 3.1, Eq. 1
 *   - front-to-back compositing of traced
 *     quantities {N, D, R, E, P}               Sec. 3.1, Eq. 2-3
 *   - light bouncing from X = O + Dt w          Sec. 3.1 "Light Bouncing"
 *   - single-bounce emission-aware render      Sec. 3.3, Eq. 5-7
 *     and its gradient (Stage 1 objective)     Sec. 3.3, Eq. 8
 *   - multi-bounce path tracing                Sec. 3.4, Eq. 9
 *   - scene edits (relighting, recolouring)    Sec. 1 and Sec. 5 results
 *   - Stage-0 objective: Nt, Dt, R, E images,
 *     their loss terms and adjoint              Sec. 3.2, Eq. 4
 *   - light baking into r (0-bounce render,
 *     its radiance gradient, PQ-L1 loss, Adam)  Sec. 3.4 "Light Baking", Eq. 10
 *   - path tracing with emitter sampling and
 *     multiple importance sampling             Sec. 5 and Appendix D (proposed there)
 *   - geometric edits: selection, rigid
 *     motion, deletion, duplication, tree cost  Sec. 1 and Sec. 5
 *
 * Conventions for every call:
 *   - Plain C. No exceptions cross the boundary; every entry point returns
 *     an eag_status and, on failure, sets a thread-local message readable
 *     with eag_last_error().
 *   - "device" pointers are HIP device memory on the current device, owned
 *     by the caller (the Python binding allocates them as torch tensors).
 *     "host" pointers are ordinary host memory. The library never calls
 *     hipMalloc/hipFree; every buffer it needs is a caller-provided
 *     workspace whose size a *_bytes query returns.
 *   - Every compute call is asynchronous on the given HIP stream
 *     (hipStream_t passed as void*; NULL = default stream) unless stated.
 *     Input buffers must stay alive until the stream reaches the call.
 *   - Asynchronous device faults surface as EAG_ERR_DEVICE from a later
 *     call; host-side validation errors return EAG_ERR_INVALID_ARGUMENT and
 *     launch nothing. Errors only the kernels can see reach a later call the
 *     same way, through a word of mapped host memory the library allocates
 *     once per process: a hit farther than the order key's last depth bucket
 *     (max_bucket * depth_quantum, with 64 - 2 ceil(log2 n) bucket bits; 32 m
 *     at 2^23 surfels and the default quantum) marks that launch's results
 *     invalid, and the next call returns EAG_ERR_DEVICE asking for a larger
 *     depth_quantum.
 *   - Arrays are component-major (structure of arrays) float32:
 *     a "[3][n]" array holds x[0..n), then y[0..n), then z[0..n).
 */
#ifndef EAG_H
#define EAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EAG_ABI_VERSION 2u

typedef enum {
  EAG_OK = 0,
  EAG_NOT_READY = 1,
  EAG_ERR_INVALID_ARGUMENT = -1,
  EAG_ERR_WORKSPACE_TOO_SMALL = -2,
  EAG_ERR_OUT_OF_BUDGET = -3,
  EAG_ERR_DEVICE = -4,
  EAG_ERR_CANCELLED = -5,
  EAG_ERR_UNKNOWN_TICKET = -6,
  EAG_ERR_INTERNAL = -7
} eag_status;

/* Message of the last non-OK status returned on this thread (never NULL). */
const char* eag_last_error(void);
uint32_t eag_abi_version(void);

/* ------------------------------------------------------------------------
 * Scene: n surfels, borrowed device arrays (Sec. 3.1: centre p, tangent
 * scales s_u, s_v, orientation quaternion q, opacity sigma; Eq. 3: linear
 * radiance r, emissive term e in [0,1], diffuse albedo rho).
 * ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;                 /* number of surfels, 1 <= n <= 2^23            */
  const float* pos;          /* device [3][n] centre p                        */
  const float* rot;          /* device [4][n] quaternion (w,x,y,z), |q| > 0   */
  const float* scale;        /* device [2][n] s_u, s_v > 0                    */
  const float* opacity;      /* device [n] sigma in [0,1); 0 = deleted        */
  const float* albedo;       /* device [3][n] rho                             */
  const float* radiance;     /* device [3][n] r (emission / radiance cache)   */
  const float* emissive;     /* device [n] e                                  */
} eag_surfels;

/* Gradients with the same shapes as the inputs; accumulated with +=, the
 * caller zeroes them. The emissive term e receives no gradient (it enters the
 * single-bounce map only through the threshold of Eq. 5). */
typedef struct {
  float* pos;                /* device [3][n] */
  float* rot;                /* device [4][n] (w.r.t. the unnormalised q) */
  float* scale;              /* device [2][n] */
  float* opacity;            /* device [n]    */
  float* albedo;             /* device [3][n] */
  float* radiance;           /* device [3][n] */
} eag_surfel_grads;

/* Pinhole camera with vertical field of view; image row 0 is the top. */
typedef struct {
  float eye[3], look_at[3], up[3];
  float vfov_deg;            /* (0, 180) */
  int32_t width, height;     /* >= 1 */
} eag_camera;

enum {
  EAG_JITTER = 1u,               /* jitter camera rays inside the pixel (Philox segment word 0xffffffff) */
  EAG_ADDITIVE_EMISSION = 2u,    /* test mode: L_o = L_e + L_r at every hit (first line of Eq. 5)       */
  EAG_DETACH_BOUNCE = 4u         /* adjoint: hold bounce origin X and direction w' constant             */
};

/* Parameters of tracing and rendering. eag_default_params fills the
 * defaults in brackets. */
typedef struct {
  int32_t spp;              /* samples per pixel [4] (Eq. 7 and Eq. 9 n_spp)                 */
  int32_t max_depth;        /* max diffuse reflections per path [5] (Eq. 9 bounce limit);   */
                            /* a path traces at most max_depth + 1 segments, <= 64           */
  int32_t rr_start;         /* Russian roulette once depth >= rr_start; 0 = off [3]           */
  float tau_E;              /* emitter threshold on composited E [0.1] (Eq. 5)                */
  float T_min;              /* compositing stops after T < T_min [1e-4] (Sec. 3.1)            */
  float t_min;              /* minimum hit distance [1e-3]                                    */
  float k_sigma;            /* accept iff u^2+v^2 <= k_sigma^2 [3]                            */
  float depth_quantum;      /* order key floor(t/dq) then surfel index [2^-13]; must be 0 or  */
                            /* a power of two; 0 = exact (t, index) order (n <= 65536)        */
  int32_t kbuf;             /* k-buffer depth, must be 16                                     */
  uint32_t camera_id;       /* 4th Philox counter word (camera c of a batch uses id + c)      */
  uint64_t seed;            /* Philox key [0]                                                 */
  uint32_t flags;           /* EAG_* flags [0]                                                */
  uint32_t reserved;
} eag_trace_params;

void eag_default_params(eag_trace_params* p);

/* ------------------------------------------------------------------------
 * Acceleration structure: a BVH over the surfels' k_sigma ellipse bounds
 * (63-bit Morton order, then locally-ordered agglomerative clustering of
 * the sorted boxes), collapsed into a 4-wide tree for traversal. The paper's implementation
 * uses an OptiX acceleration structure (Sec. 5 "Implementation Details");
 * gfx950 has no ray-tracing units, so this one is built and traversed by
 * hand-written kernels.
 *
 * The BVH stores a snapshot of the geometry (p, q, s, sigma) taken at build
 * or refit time; renders read geometry from it and attributes (rho, r, e)
 * from the eag_surfels passed to each call. After changing geometry, call
 * eag_refit_bvh (same n, same topology) or rebuild.
 * ------------------------------------------------------------------------ */
typedef struct eag_bvh eag_bvh;   /* opaque host handle; node storage is in caller memory */

typedef struct {
  int64_t n;                 /* surfels                              */
  int32_t max_depth;         /* deepest leaf (root = 0)              */
  int32_t root;              /* root reference (>= 0 internal node; <0: leaf ~ref) */
  float lo[3], hi[3];        /* scene bounds of the surfel boxes     */
  const void* nodes;         /* device: (n-1) internal nodes, 64 B each:  */
                             /*   float lo0[3], hi0[3], lo1[3], hi1[3]; int32 child0, child1, pad[2] */
                             /*   child >= 0: internal node, child < 0: leaf at sorted position ~child */
  const void* records;       /* device: n geometry records, 48 B each, in sorted (Morton) order */
  const int32_t* perm;       /* device [n]: sorted position -> surfel index */
  const void* nodes4;        /* device: the 4-wide tree traversed by the tracer, 128 B per node: */
                             /*   float box[4][6] (lo.xyz hi.xyz); int32 ref[4] (>= 0 node, < 0 leaf ~pos, */
                             /*   0x7fffffff empty); int32 src[4] (binary-tree origin of each child) */
  int32_t n_nodes4;          /* nodes in nodes4; node 0 is the root */
  int32_t depth4;            /* levels of the 4-wide tree */
} eag_bvh_info;

size_t eag_bvh_bytes(int64_t n);
size_t eag_build_workspace_bytes(int64_t n);
/* Build. Stream-ordered and asynchronous: the call enqueues the build on
 * `stream` and returns; depths, node count and bounds stay on the device
 * (eag_bvh_get_info waits for them). bvh_mem: device, >= eag_bvh_bytes(n),
 * 256-B aligned, owned by the caller and referenced by the handle until
 * eag_bvh_destroy. ws: device scratch, in use until the stream reaches the
 * end of the build. Any tree the build can make fits the traversal stack
 * (at most 63 + ceil(log2 n) levels), so nothing is checked after it. */
eag_status eag_build_bvh(const eag_surfels* s, void* bvh_mem, size_t bvh_bytes,
                         void* ws, size_t ws_bytes, void* stream, eag_bvh** out);
/* Recompute frames, records and node bounds after a geometry edit that keeps
 * n; topology is kept (Morton order of the build). Stream-ordered and
 * asynchronous, like the build. */
eag_status eag_refit_bvh(eag_bvh* bvh, const eag_surfels* s, void* ws, size_t ws_bytes, void* stream);
/* Waits for the last build or refit of the handle (host-blocking, the one
 * BVH call that is) and reports its shape and bounds. */
eag_status eag_bvh_get_info(const eag_bvh* bvh, eag_bvh_info* out);
void eag_bvh_destroy(eag_bvh* bvh);

/* ------------------------------------------------------------------------
 * Tracing (Sec. 3.1, Eq. 1-3): blend every surfel on each ray front to back
 * through a 16-entry k-buffer, in order of the key (floor(t/dq), index),
 * stopping after the first hit with T < T_min.
 * ------------------------------------------------------------------------ */
size_t eag_trace_workspace_bytes(int64_t n_surfels);
/* origins, dirs: device double [3][n_rays], dirs unit length (the tracer's
 * ray geometry is double precision throughout).
 * out: device [12][n_rays] = Nt(3), Dt, R(3), E, P(3), A (Nt = N/|N|, Dt = D/A;
 *      all zero for a miss).
 * hit_idx: nullable device [n_rays][max_hits] surfel indices in blending order;
 * hit_count: nullable device [n_rays] number of blended hits (may exceed
 * max_hits; only the first max_hits are written).
 * stats: nullable device [n_rays][3] traversal statistics per ray: k-buffer
 * rounds, candidate surfel tests, internal nodes visited. */
eag_status eag_trace_rays(const eag_bvh* bvh, const eag_surfels* s, const eag_trace_params* p,
                          int64_t n_rays, const double* origins, const double* dirs, float* out,
                          int32_t* hit_idx, int32_t* hit_count, int32_t max_hits, int32_t* stats,
                          void* ws, size_t ws_bytes, void* stream);

/* Set-up for callers that cannot allocate: allocates the library's status
 * word (once per process) and looks up the no-allocation scratch of the
 * current device. Call it once on each device, with that device current,
 * before eag_trace_rays_noalloc; idempotent. */
eag_status eag_init(void);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): eag_trace_rays without
 * a workspace, allocating nothing. Its scratch (the scene's packed attribute
 * records) is a static device array of EAG_NOALLOC_MAX_SURFELS records per
 * device: scenes of more surfels are rejected with EAG_ERR_INVALID_ARGUMENT,
 * and so are calls on a device eag_init has not set up. Every call on a
 * device shares that device's array, so calls that overlap on one device
 * (other streams, other threads) race; each call rewrites the records it
 * reads. Arguments and results as eag_trace_rays. */
#define EAG_NOALLOC_MAX_SURFELS (1 << 18)
eag_status eag_trace_rays_noalloc(const eag_bvh* bvh, const eag_surfels* s, const eag_trace_params* p,
                                  int64_t n_rays, const double* origins, const double* dirs, float* out,
                                  int32_t* hit_idx, int32_t* hit_count, int32_t max_hits, int32_t* stats,
                                  void* stream);

/* ------------------------------------------------------------------------
 * Single-bounce emission-aware render (Sec. 3.3, Eq. 5-7): per pixel, the
 * camera segment through the pixel centre gives (Nt, Dt, R, E, P, A); a miss
 * renders 0, E > tau_E renders R, otherwise P * (1/spp) sum_s R(w'_s) with w'_s
 * cosine-sampled about Nt from X = O + Dt w (Philox counter (pixel, s, 0,
 * camera_id + c)). Secondary segments blend r without an emitter test (the
 * radiance cache).
 * ------------------------------------------------------------------------ */
/* Forward state kept for the backward pass: per pixel EAG_FWD_PIXEL_FLOATS
 * floats (as doubles: Nt(3), Dt, |N|, A, R(3), P(3); then float E and the
 * branch 0 miss / 1 emitter / 2 reflect, and two pad floats), followed by
 * the R of every secondary sample as doubles [n_cams][H][W][spp][3].
 * Total floats: n_cams*H*W*(EAG_FWD_PIXEL_FLOATS + 6*spp). */
#define EAG_FWD_PIXEL_FLOATS 28
int64_t eag_fwd_state_floats(const eag_camera* cams, int32_t n_cams, const eag_trace_params* p);
/* Workspace of eag_render_single_bounce: packed attributes, forward state,
 * per-sample adjoints, double gradient accumulators, a work counter and the
 * hit list of the persistent secondary passes (1 KiB per lane of the
 * persistent grid, which depends on the current device: 128 MiB on MI355X).
 * Returns 0 and sets the last error if the device cannot be queried. */
size_t eag_render_workspace_bytes(int64_t n_surfels, const eag_camera* cams, int32_t n_cams,
                                  const eag_trace_params* p);
/* Workspace of eag_single_bounce_backward: the render workspace plus the
 * per-hit gradient records of the adjoint passes: 64 B for up to 20 hits
 * per (pixel, sample) of one batch of up to 8 cameras, at most 2^27 records
 * (8 GiB), and per-surfel counters. Hits beyond the records are added with
 * atomics instead, so the result does not depend on the size; the speed
 * does. Returns 0 and sets the last error if the device cannot be queried. */
size_t eag_backward_workspace_bytes(int64_t n_surfels, const eag_camera* cams, int32_t n_cams,
                                    const eag_trace_params* p);
/* cams: host [n_cams], all the same width and height.
 * rgb: device [n_cams][H][W][3].
 * fwd_state: nullable device buffer of eag_fwd_state_floats() floats. */
eag_status eag_render_single_bounce(const eag_bvh* bvh, const eag_surfels* s, const eag_camera* cams,
                                    int32_t n_cams, const eag_trace_params* p, float* rgb, float* fwd_state,
                                    void* ws, size_t ws_bytes, void* stream);
/* Exact reverse of eag_render_single_bounce with every discrete decision of
 * the forward pass held fixed (hit sets, order, stopping hit, normal signs,
 * emitter branch); includes the chain through X (via Dt) and w' (via Nt and
 * the hemisphere frame) unless EAG_DETACH_BOUNCE. Hit lists are recomputed,
 * not stored. dL_drgb: device [n_cams][H][W][3]; fwd_state from the forward
 * call with the same arguments; ws of eag_backward_workspace_bytes() bytes.
 * Per-hit contributions, rounded to float, are summed in double precision in
 * the workspace, through per-hit records grouped by surfel (a sum's error is
 * about 2^-24 of the sum of its terms' magnitudes at most), and added once to
 * `grads` (grads += sum; the caller zeroes them for a fresh gradient). */
eag_status eag_single_bounce_backward(const eag_bvh* bvh, const eag_surfels* s, const eag_camera* cams,
                                      int32_t n_cams, const eag_trace_params* p, const float* dL_drgb,
                                      const float* fwd_state, const eag_surfel_grads* grads,
                                      void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Multi-bounce path tracing (Sec. 3.4, Eq. 9) in a persistent wavefront
 * kernel. Per path: miss -> 0; E > tau_E -> add beta*R and stop; depth ==
 * max_depth -> discard; else beta *= P, cosine-sample w' (Philox counter
 * (pixel, sample, depth, camera_id)), continue from X; Russian roulette when
 * the new depth >= rr_start: q = min(0.95, max beta), survive iff u2 < q,
 * beta /= q.
 * accum: device int64 [H][W][3] running sums in fixed point (value *
 * EAG_ACCUM_SCALE, rounded to nearest); the sums are independent of launch
 * order and of how samples are split across calls. Samples
 * [sample_begin, sample_begin + sample_count) are added.
 * counters: nullable device uint64 [6] += {segments traced, paths started,
 * k-buffer rounds, candidate surfel tests, blended hits, BVH nodes visited}.
 * ------------------------------------------------------------------------ */
#define EAG_ACCUM_SCALE 4294967296.0 /* 2^32 */
/* Workspace of eag_path_trace: packed attributes (32 B per surfel), a work
 * counter, and a hit list of 1 KiB per lane of the persistent grid, which
 * depends on the current device (256 CUs x 512 lanes on MI355X: 128 MiB).
 * Returns 0 and sets the last error if the device cannot be queried. */
size_t eag_path_trace_workspace_bytes(int64_t n_surfels);
eag_status eag_path_trace(const eag_bvh* bvh, const eag_surfels* s, const eag_camera* cam,
                          const eag_trace_params* p, uint32_t sample_begin, uint32_t sample_count,
                          int64_t* accum, uint64_t* counters, void* ws, size_t ws_bytes, void* stream);
/* rgb[i] = accum[i] / (EAG_ACCUM_SCALE * total_spp) for i < 3*n_pixels (device arrays). */
eag_status eag_accum_resolve(const int64_t* accum, int64_t n_pixels, int32_t total_spp, float* rgb,
                             void* stream);

/* ------------------------------------------------------------------------
 * Path tracing with emitter sampling: next-event estimation on emissive
 * surfels combined with the cosine sampling above by multiple importance
 * sampling, the remedy for small emitters that Sec. 5 and Appendix D
 * (Discussion) propose without fixing an estimator. The estimator built
 * here has the expectation of eag_path_trace:
 *   emitters    surfels with e > tau_E and opacity > 0;
 *   selection   emitter j with probability w_j / W, w_j = opacity s_u s_v
 *               (mean of r + e), by inversion of the inclusive prefix sums
 *               on u0 (the first j whose sum exceeds u0 W);
 *   point       uniform on the j's k_sigma ellipse from u1, u2 (radius
 *               k sqrt(u1), angle 2 pi u2);
 *   light pdf   p_l(X, w) = sum over the emitter ellipses the ray X + d w
 *               crosses at d > 0 of rho_j d^2 / |w . n_j|, rho_j =
 *               opacity (mean of r + e) / (pi k^2 W);
 *   weights     power heuristic against p_b = max(0, w . Nt) / pi: at each
 *               reflecting vertex the light segment from X towards the point
 *               adds beta R p_b p_l / (p_b^2 + p_l^2) if it passes the emitter
 *               test (beta after the vertex's P, before Russian roulette); a
 *               cosine-sampled segment k >= 1 that passes it adds
 *               beta R p_b^2 / (p_b^2 + p_l^2); the camera segment adds beta R.
 * The light sample after segment k uses Philox counter (pixel, sample,
 * 2^31 + k, camera_id); everything else is eag_path_trace's.
 * ------------------------------------------------------------------------ */
typedef struct eag_emitters eag_emitters;   /* opaque host handle; storage in caller memory */
/* Device memory of a table for a scene of n_surfels (sized for every
 * surfel being an emitter), and the workspace of its build. */
size_t eag_emitters_bytes(int64_t n_surfels);
size_t eag_emitters_workspace_bytes(int64_t n_surfels);
/* Builds the table of s for p->tau_E (>= 0) and p->k_sigma (<= 3, the
 * extent of the tree's boxes): compacted emitter attributes, prefix sums,
 * densities and a tree over the emitters. mem (256-B aligned, >=
 * eag_emitters_bytes) is referenced by the handle until
 * eag_emitters_destroy; ws only during the call. Synchronises `stream`.
 * The table is a copy: rebuild it after editing the scene.
 * cell: 0 selects emitters by power alone, as above. A power of two in
 * [2^-10, 2^10] (scene units) selects by cells instead. Emitters are grouped
 * by the cube of that side holding their centre (floor of the float32 centre
 * over cell, per axis), in the order (cell, surfel index). At a vertex X, a
 * cell is chosen with probability I_c / sum I over the cells, where
 * I_c = W_c / max(|X - m_c|^2, cell^2), W_c is the cell's summed w_j and m_c
 * its centre; inversion on u0 over the cells in order picks it. An emitter
 * of the cell is then chosen with probability w_j / W_c, by inversion on u3
 * (the fourth word of the light sample's Philox counter). rho_j becomes
 * (I_c / sum I) opacity (mean of r + e) / (pi k^2 W_c). Emitters near the
 * vertex are drawn more often, and those in other rooms seldom. Centres must
 * satisfy |coordinate| / cell < 2^20 (cell keys hold 21 bits per axis); the
 * selection at each vertex loops over all cells. */
eag_status eag_build_emitters(const eag_surfels* s, const eag_trace_params* p, float cell, void* mem,
                              size_t mem_bytes, void* ws, size_t ws_bytes, void* stream, eag_emitters** out);
/* count: emitters in the table; total_weight: W (0 when there are none);
 * n_cells: cells of the selection by cells (0 for selection by power). Each
 * output is nullable. */
eag_status eag_emitters_get_info(const eag_emitters* em, int64_t* count, double* total_weight, int32_t* n_cells);
void eag_emitters_destroy(eag_emitters* em);
/* Workspace of eag_path_trace_mis for its fastest launches: eag_path_trace's,
 * plus a queue for the contributions that wait for their light pdf (96 B per
 * entry, W H (max_depth + 1) entries per sample, for 4 samples per launch).
 * A smaller workspace also works: the call then launches as many samples at
 * a time as its queue holds, and fails only when one sample does not fit.
 * 0 for invalid arguments. */
size_t eag_path_trace_mis_workspace_bytes(int64_t n_surfels, const eag_camera* cam, const eag_trace_params* p);
/* As eag_path_trace (same accumulator and sample ranges) with the estimator
 * above; ws: eag_path_trace_mis_workspace_bytes. em must come from the same
 * scene (same surfel count) and the same tau_E and k_sigma as p;
 * EAG_ADDITIVE_EMISSION is rejected. A table without emitters gives
 * eag_path_trace's values. counters: nullable device uint64 [7]: the six of
 * eag_path_trace, then the number of queued contributions dropped because
 * the queue was full (0 unless a launch queues more than one entry per
 * segment: the image then lacks them). */
eag_status eag_path_trace_mis(const eag_bvh* bvh, const eag_surfels* s, const eag_emitters* em,
                              const eag_camera* cam, const eag_trace_params* p, uint32_t sample_begin,
                              uint32_t sample_count, int64_t* accum, uint64_t* counters, void* ws,
                              size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Scene edits (the paper's relighting and material edits, Sec. 1, Sec. 5).
 * Attribute edits write the caller's arrays in place and need no refit.
 * ------------------------------------------------------------------------ */
enum {
  EAG_EDIT_SET_RADIANCE = 1,    /* r[i] = value[0..2]                         */
  EAG_EDIT_SCALE_RADIANCE = 2,  /* r[i] *= value[0..2] (0 switches lights off) */
  EAG_EDIT_SET_ALBEDO = 3,      /* rho[i] = value[0..2]                       */
  EAG_EDIT_SET_EMISSIVE = 4,    /* e[i] = value[0]                            */
  EAG_EDIT_TRANSFORM = 5        /* rigid motion (server only; eag_move_surfels
                                   applies it to caller arrays): value[0..3] =
                                   unit quaternion r (w, x, y, z), value[4..6] =
                                   pivot, value[7..9] = translation t;
                                   p -> R(r)(p - pivot) + pivot + t, q -> r (x) q */
};
typedef struct {
  int32_t kind;
  const int32_t* idx;           /* device [count] surfel indices; indices outside
                                   [0, n) are skipped */
  int64_t count;
  float value[12];              /* per kind, as above; the rest unused */
} eag_edit;
typedef struct {
  int64_t n;
  float* albedo;                /* device [3][n] */
  float* radiance;              /* device [3][n] */
  float* emissive;              /* device [n]    */
} eag_surfel_attrs;
eag_status eag_apply_edit(const eag_edit* e, const eag_surfel_attrs* a, void* stream);

/* ------------------------------------------------------------------------
 * Geometric edits (Sec. 1 and Sec. 5: moving, importing and deleting
 * objects). Selection by box, rigid motions, deletion and duplication of
 * surfels, and the surface-area cost of a tree, by which a caller chooses
 * between eag_refit_bvh (same surfels, moved) and a new eag_build_bvh
 * (after duplication the surfel count changes, and only a build will do).
 * r: host float[4], a rotation quaternion (w, x, y, z), normalised here;
 * pivot, t: host float[3]. A motion maps p to R(r) (p - pivot) + pivot + t
 * and q to r (x) q (Hamilton product), computed in double precision.
 * ------------------------------------------------------------------------ */
typedef struct {                /* writable surfel arrays, shapes as eag_surfels */
  int64_t n;
  float *pos, *rot, *scale, *opacity, *albedo, *radiance, *emissive;
} eag_surfels_out;
size_t eag_select_workspace_bytes(int64_t n_surfels);
/* The surfels whose centre lies in the closed box [lo, hi] (host float[3]
 * each; compared in float32): idx (device int32 [n]) receives them in
 * ascending order, count (device int64) their number. */
eag_status eag_select_box(const eag_surfels* s, const float* lo, const float* hi, int32_t* idx, int64_t* count,
                          void* ws, size_t ws_bytes, void* stream);
/* Moves surfels idx[0..count) (device) of s in place (pos and rot only). */
eag_status eag_move_surfels(const eag_surfels_out* s, const int32_t* idx, int64_t count, const float* r,
                            const float* pivot, const float* t, void* stream);
/* Deletes surfels idx[0..count) of s: their opacity becomes 0. */
eag_status eag_delete_surfels(const eag_surfels_out* s, const int32_t* idx, int64_t count, void* stream);
/* dst (n = src->n + count) receives src's surfels, then copies of
 * src's surfels idx[0..count) moved by (r, pivot, t). */
eag_status eag_duplicate_surfels(const eag_surfels* src, const int32_t* idx, int64_t count, const eag_surfels_out* dst,
                                 const float* r, const float* pivot, const float* t, void* stream);
/* cost (device double) = 1 + (sum over every node of the surface areas of
 * its children's boxes) / (surface area of the root's box); 1 for a
 * one-surfel scene. ws: eag_build_workspace_bytes(n) bytes suffice. */
eag_status eag_bvh_sah_cost(const eag_bvh* bvh, double* cost, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Stage 0, the radiant scene (Sec. 3.2, Eq. 4). Per pixel, one camera ray
 * (sample 0, the pixel centre unless EAG_JITTER) and its segment's images:
 * Nt = N/|N|, Dt = D/A, R, E (Eq. 3), 8 floats per pixel in that order, all
 * 0 for a pixel that blends nothing. The objective, with weights
 * (lc, ln, ld, le):
 *   lc * mean over pixels and channels of |PQ(R) - PQ(R_gt)|
 *   ln * mean over hit pixels of (1 - Nt . N_mono)
 *   ld * mean over valid pixels of (1 - N_d . N_mono)
 *   le * mean over pixels of |E - M|
 * with PQ as for light baking. N_d, the distance normal, is the normal of
 * the points X = O + Dt W: normalize((X(x+1,y) - X(x-1,y)) x (X(x,y+1) -
 * X(x,y-1))), turned to face the camera; a pixel is valid when it and its
 * four neighbours are inside the image and hit.
 * ------------------------------------------------------------------------ */
/* Workspace of eag_render_stage0 and eag_stage0_backward: packed attributes,
 * the persistent grid's hit list, double accumulators and per-hit gradient
 * records (64 B for up to 20 hits per pixel of a batch of up to 8 cameras)
 * and per-pixel scratch. 0 and the last error if the device cannot be
 * queried. */
size_t eag_stage0_workspace_bytes(int64_t n_surfels, const eag_camera* cams, int32_t n_cams);
/* images: device [n_cams][H][W][8] (written). fwd_state: device, n_cams*H*W*
 * EAG_FWD_PIXEL_FLOATS floats (written; the camera segments' totals, kept
 * for eag_stage0_backward). */
eag_status eag_render_stage0(const eag_bvh* bvh, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                             const eag_trace_params* p, float* images, float* fwd_state, void* ws, size_t ws_bytes,
                             void* stream);
/* Workspace of eag_stage0_loss (counters and per-pixel scratch; no scene). */
size_t eag_stage0_loss_workspace_bytes(const eag_camera* cams, int32_t n_cams);
/* The objective of images (as eag_render_stage0 writes them) against
 * rgb_gt [n_cams][H][W][3], normal_mono [n_cams][H][W][3] (unit) and mask
 * [n_cams][H][W] (device float arrays); weights: host float[4] = (lc, ln,
 * ld, le). Writes loss (device double) and d_images [n_cams][H][W][8], its
 * gradient in the images (the hit mask held fixed). */
eag_status eag_stage0_loss(const float* images, const float* rgb_gt, const float* normal_mono, const float* mask,
                           const eag_camera* cams, int32_t n_cams, const eag_trace_params* p, const float* weights,
                           float* d_images, double* loss, void* ws, size_t ws_bytes, void* stream);
/* Parameter gradients of sum(d_images * images), every discrete decision of
 * the forward held fixed (hit lists, order, stopping hit, normal signs):
 * grads->pos, rot, scale, opacity, radiance and grad_emissive [n] get +=
 * (albedo is untouched; the caller zeroes the arrays for a fresh gradient).
 * fwd_state: from eag_render_stage0 with the same arguments. */
eag_status eag_stage0_backward(const eag_bvh* bvh, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                               const eag_trace_params* p, const float* d_images, const float* fwd_state,
                               const eag_surfel_grads* grads, float* grad_emissive, void* ws, size_t ws_bytes,
                               void* stream);

/* ------------------------------------------------------------------------
 * Light baking (Sec. 3.4 "Light Baking", Eq. 10): the per-surfel radiance r
 * is refitted so that the 0-bounce image (R composited along each camera
 * ray, Sec. 3.2) matches path-traced renders of the (edited) scene:
 * min_r L1(PQ(L0), PQ(Lpt)). Geometry and opacity are fixed, so the
 * blending weights of every camera ray do not depend on r and L0 is linear
 * in it. PQ is SMPTE ST 2084 on Y = max(L, 0) / 10000 (radiance read as
 * cd/m^2), its derivative taken at max(Y, 2^-24). One camera ray per pixel:
 * sample 0, the pixel centre unless EAG_JITTER.
 * ------------------------------------------------------------------------ */
typedef struct {
  float lr;                     /* step size                                     */
  float beta1, beta2;           /* moment decay rates (0.9, 0.999)               */
  float eps;                    /* added to sqrt(v_hat) (1e-15)                  */
} eag_adam;
/* Workspace of the calls below for n_cams cameras of one size: packed
 * attributes, the persistent grid's hit list (device dependent: 128 MiB on
 * MI355X), double radiance-gradient accumulators, and the image and image
 * gradient of eag_bake_step. 0 and the last error if the device cannot be
 * queried. */
size_t eag_bake_workspace_bytes(int64_t n_surfels, const eag_camera* cams, int32_t n_cams);
/* 0-bounce image. rgb: device [n_cams][H][W][3] (written). Only the
 * geometry, opacity and radiance of s are read. */
eag_status eag_render_zero_bounce(const eag_bvh* bvh, const eag_surfels* s, const eag_camera* cams,
                                  int32_t n_cams, const eag_trace_params* p, float* rgb,
                                  void* ws, size_t ws_bytes, void* stream);
/* Radiance gradient of sum(dL_drgb * L0): every blended hit i of a pixel
 * adds w_i * dL to its surfel's row (w_i = T_{i-1} alpha_i), summed in
 * double precision, then grad_radiance += sum. dL_drgb: device
 * [n_cams][H][W][3]; grad_radiance: device [3][n] (caller zeroes it for a
 * fresh gradient). Pixels whose dL is zero are not traced. */
eag_status eag_zero_bounce_backward(const eag_bvh* bvh, const eag_surfels* s, const eag_camera* cams,
                                    int32_t n_cams, const eag_trace_params* p, const float* dL_drgb,
                                    float* grad_radiance, void* ws, size_t ws_bytes, void* stream);
/* loss = mean over the n_values values of |PQ(rgb) - PQ(target)| (device
 * double, written), dL_drgb = its derivative in rgb (device, n_values,
 * written; 0 where the two are equal). */
eag_status eag_bake_loss(const float* rgb, const float* target, int64_t n_values, float* dL_drgb,
                         double* loss, void* stream);
/* One Adam update with bias correction (step counts from 1) of the n
 * values of param, then param clamped at 0: m, v are the caller's first
 * and second moment arrays (device, n each, zero before the first step). */
eag_status eag_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, const eag_adam* a,
                         int32_t step, void* stream);
/* One baking iteration over n_cams views: 0-bounce render, loss against
 * targets (device [n_cams][H][W][3], e.g. resolved path-traced images),
 * radiance gradient and the Adam update of radiance, which must be
 * s->radiance (device [3][n], updated in place; m, v as for eag_adam_step).
 * loss: device double, written with the loss before the update. */
eag_status eag_bake_step(const eag_bvh* bvh, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                         const eag_trace_params* p, const float* targets, float* radiance, float* m, float* v,
                         const eag_adam* a, int32_t step, double* loss, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a resident scene answering path-tracing requests with continuous
 * batching. A host scheduler thread admits requests while their fixed-point
 * accumulators fit the arena and a slot is free, and each launch of the
 * multi-request persistent kernel draws paths from the live requests, the
 * one with the least work left first, so requests that arrive while others
 * run join the next launch and short ones do not wait behind long ones. Edits are
 * ordered with respect to later submits: each request renders the scene
 * version current at its submit; attribute edits create a new version
 * (copy-on-write attributes); geometry is shared, so a geometric edit
 * (a rigid motion with a BVH refit) first lets earlier requests finish.
 * ------------------------------------------------------------------------ */
typedef struct eag_server eag_server;
typedef struct {
  void* arena;                  /* device memory owned by the caller            */
  size_t arena_bytes;
  int32_t max_live_requests;    /* slots, 1..8                                  */
  int64_t paths_per_launch;     /* work quantum of one launch (all live requests) */
  void* stream;                 /* stream the server launches on                */
} eag_server_config;
typedef struct {
  eag_camera cam;
  eag_trace_params params;      /* spp, max_depth, rr_start, seed, camera_id ... */
  float* out_rgb;               /* device [H][W][3], written when done           */
} eag_request;
typedef struct {
  int32_t status;               /* EAG_OK, EAG_NOT_READY, or an error          */
  uint32_t scene_version;
  double t_submit, t_admit, t_done;   /* seconds, host monotonic clock           */
  uint64_t paths;
} eag_result;
/* Bytes of arena needed for a scene of n surfels with `versions` attribute
 * versions, on the current device (the arena holds the path tracer's hit
 * list, whose size depends on the device; 0 and the last error if it cannot
 * be queried). */
size_t eag_serve_arena_bytes(int64_t n, int32_t versions, size_t request_bytes);
/* Copies the scene into the arena and builds the BVH (synchronous). */
eag_status eag_serve_create(const eag_surfels* s, const eag_server_config* cfg, eag_server** out);
eag_status eag_serve_submit(eag_server* srv, const eag_request* req, uint64_t* ticket);  /* non-blocking */
/* Queues an edit, ordered with respect to earlier and later submits (non-
 * blocking). e->idx is a device array that the server reads when it applies
 * the edit, on its stream: the caller keeps it unchanged until the ticket
 * reports done. Attribute kinds make a new copy-on-write attribute version.
 * EAG_EDIT_TRANSFORM moves the resident geometry, which all versions share,
 * and refits the BVH: it waits until every request submitted before it has
 * completed (requests submitted after it wait behind it), then applies the
 * motion, refits, and makes a new version. */
eag_status eag_serve_edit(eag_server* srv, const eag_edit* e, uint64_t* ticket);
eag_status eag_serve_poll(eag_server* srv, uint64_t ticket, eag_result* out);           /* non-blocking */
eag_status eag_serve_cancel(eag_server* srv, uint64_t ticket);
eag_status eag_serve_destroy(eag_server* srv);  /* drains, stops the scheduler thread */

#ifdef __cplusplus
}
#endif
#endif /* EAG_H */
