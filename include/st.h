/*
 * st.h -- C ABI of the synchronized blobtree tracer for MI355X (gfx950).
 *
 * The library ray-casts a blobtree (a binary tree whose leaves are primitives
 * and whose inner nodes are CSG operators) and writes a G-buffer of hit depth
 * and unit normal per pixel: for each pixel ray r(t) it finds the first t with
 * f(r(t)) = 0 (the iso-surface problem statement of "Implicit volume
 * visualization", Section 2.2 of Zanni 2023, "Synchronized-tracing of implicit
 * surfaces"), with deferred shading left to the caller (Section "GPU runtime
 * statistics").  The pipeline is the paper's: a per-screen-tile A-buffer of
 * primitive volumes of interest (Section 6), then per-tile synchronized sphere
 * tracing of subfrustums with a bottom-up pruned tree (Sections 7 and 8,
 * Algorithms 2 and 3).
 *
 * Conventions for every call:
 *  - All functions return st_status; no C++ exception crosses the ABI.  On
 *    failure, st_last_error() returns a thread-local message.
 *  - "device" pointers are HIP device allocations on the current device;
 *    "host" pointers are ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it; calls are asynchronous unless stated otherwise.
 *  - Handles are not thread safe: one thread at a time per st_scene.
 */
#ifndef ST_H
#define ST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ST_OK = 0,
    ST_E_INVALID = 1,   /* bad argument: NULL, NaN/inf parameter, bad camera or tuning */
    ST_E_TREE = 2,      /* malformed blobtree */
    ST_E_CAPACITY = 3,  /* a fixed capacity of the library was exceeded */
    ST_E_NOMEM = 4,     /* device or host allocation failed */
    ST_E_DEVICE = 5,    /* a HIP call failed; st_last_error() has HIP's message */
    ST_E_STALE = 6      /* the A-buffer was built for another camera/scene version */
} st_status;

/* Node kinds.  Primitives are exact signed distances (Lipschitz 1), as the
 * paper requires of primitives that get volumes of interest (Section 6.1).
 * Operators: sharp CSG min / max / max(f0,-f1) (Section 2.1) and the compact
 * smooth operators of Section 5 (the piecewise operator G_op built on the
 * polynomial blends g, with the blend radius interpolated by b_r). */
enum {
    ST_SPHERE = 0,   /* p[0..2] centre, p[3] radius > 0 */
    ST_BOX = 1,      /* p[0..2] centre, p[3..5] half extents > 0,
                        p[6..9] rotation quaternion (w,x,y,z), non-zero; the
                        box axes are the columns of its rotation matrix */
    ST_CAPSULE = 2,  /* p[0..2] a, p[3..5] b, p[6] radius > 0 */
    ST_TORUS = 3,    /* p[0..2] centre, p[3] major radius R > 0, p[4] minor
                        radius r > 0, p[5..8] rotation quaternion (w,x,y,z),
                        non-zero; the ring lies in the local x-z plane around
                        the local y axis (the column of the rotation) */
    ST_CYLINDER = 4, /* capped cylinder: p[0..2] centre, p[3] radius > 0,
                        p[4] half height > 0, p[5..8] rotation quaternion;
                        its axis is the local y axis */
    ST_CONE = 5,     /* capped cone: p[0..2] centre, p[3] bottom radius >= 0
                        (the disk at local y = -p[4]), p[4] half height > 0,
                        p[5..8] rotation quaternion, p[9] top radius >= 0 (at
                        y = +p[4]); p[3] + p[9] > 0; axis the local y axis */
    ST_UNION = 16,   /* sharp union, no parameters */
    ST_INTER = 17,   /* sharp intersection */
    ST_DIFF = 18,    /* sharp difference left \ right */
    ST_SUNION = 19,  /* compact smooth union: p[0] blend radius k > 0,
                        p[1] operator range d_o (<= 0: d_o = 7k/6) */
    ST_SINTER = 20,  /* compact smooth intersection, same parameters */
    ST_SDIFF = 21    /* compact smooth difference, same parameters */
};

/* One blobtree node as the caller describes it (any node order). */
typedef struct {
    uint32_t kind;
    int32_t left, right;   /* child indices into the caller's array; -1 for primitives */
    float p[16];           /* parameters, layout per kind above */
} st_node;

/* Pinhole camera.  Pixel (i, j) -- column i, row j, row 0 at the top -- has
 * the ray through its centre: x = (2(i+1/2)/W - 1) tan(fov/2) W/H,
 * y = (1 - 2(j+1/2)/H) tan(fov/2), dir = normalize(x right + y up + fwd),
 * fwd = normalize(target - eye), right = normalize(fwd x up_hint),
 * up = right x fwd.  t is the distance along the unit direction. */
typedef struct {
    float eye[3], target[3], up[3];
    float vfov_deg;        /* in (0, 180) */
    int32_t width, height; /* > 0 */
} st_camera;

enum { ST_STEP_PLAIN = 0, ST_STEP_OVERRELAX = 1, ST_STEP_LEARNED = 2, ST_STEP_SEGMENT = 3 };

/* Tuning of the A-buffer build and the tracer.  st_default_tuning() fills the
 * paper's defaults where it gives one (Section 10, Implementation details). */
typedef struct {
    int32_t tile;          /* A-buffer tile edge in pixels: 8, 16 or 32 */
    int32_t max_active;    /* per-wave capacity of active primitives held on
                              chip (the paper's M_overlap, 96); tiles whose
                              volumes of interest overlap more at some depth
                              run on a wider-capacity path, never fail */
    float sub_depth;       /* fetch-ahead depth d as a fraction of the scene's
                              view-depth span (paper: 1/20) */
    int32_t max_new;       /* new primitives fetched per subfrustum, >= 1 (values
                              above 4096 act as 4096)
                              (paper: 6) */
    float eps;             /* minimum step: the shortest probe, scene units */
    int32_t max_steps;     /* field evaluations per ray for stepping */
    int32_t refine_iters;  /* bracket refinement iterations after a crossing */
    int32_t step_mode;     /* ST_STEP_*: PLAIN, the safe step f/L; OVERRELAX,
                              the step omega f/L accepted only when the spheres
                              of radius f/L at both ends overlap, else the plain
                              step (Section 10, Ray processing); LEARNED, the
                              same test with omega from the step model
                              (st_set_step_model; not in the paper); SEGMENT,
                              segment tracing (Galin et al. 2020, which the
                              paper names as the more robust replacement of
                              its global Lipschitz constant, Section 2 and
                              Section 10): the step is the longer of f/L and
                              min(c, f/lam), lam a bound on the field's
                              derivative along the ray over the candidate
                              segment [t, t+c] (compact operators whose two
                              operands cannot both reach d_o on it count as
                              min/max), and the next candidate is twice the
                              step */
    float omega;           /* over-relaxation factor for ST_STEP_OVERRELAX, in
                              [1, 4] (paper: 1.7) */
    float lipschitz;       /* 0: proven bound of each pruned view; > 0: this
                              fixed global bound (paper: 1.45, not proven) */
    int32_t keep_all_entries; /* 0 (default): drop, at binning, the entries
                              of primitives that cannot reach the root for any
                              subset of their tile's list (every subfrustum
                              view stays the same; not in the paper);
                              1: keep every entry whose volume of interest a
                              pixel-centre ray of the tile meets */
    float probe_step;      /* where the safe step f/L falls below this (scene
                              units; values below eps act as eps) the ray
                              probes forward instead: by 3/4 of the secant
                              estimate of the distance to the root while f
                              falls, by twice the last probe while f rises;
                              at least eps, at most 4x the last probe and
                              8x probe_step, never less than f/L; a sign
                              change is refined by regula falsi.  A stretch
                              of negative field at least 8x probe_step long
                              is never stepped over.  The paper steps by
                              max(f/L, minimum step) (Section 10, Ray
                              processing); default 1e-3 */
    int32_t reserved[4];
} st_tuning;

/* Counters of one st_trace call (all 64-bit). */
typedef struct {
    uint64_t rays, hits, unconverged;
    uint64_t field_evals;     /* evaluations of the pruned field at one point:
                                 steps, probes, refinements, learned-step
                                 checks; a value+gradient evaluation counts 1 */
    uint64_t grad_evals;      /* value+gradient evaluations (normals) */
    uint64_t node_evals[4];   /* by node class: sphere, box-frame primitive
                                 (box, torus, cylinder), capsule, operator */
    uint64_t grad_node_evals[4];
    uint64_t steps;           /* stepping evaluations (no refinement/gradient) */
    uint64_t subfrustums;     /* (wave, subfrustum) pairs processed */
    uint64_t empty_views;     /* subfrustums whose pruned root is unused (no surface) */
    uint64_t view_nodes;      /* sum of pruned-view sizes over subfrustums */
    uint64_t abuffer_entries; /* A-buffer entries the tracer reads (kept by
                                 the tile-level pruning) */
    uint64_t max_list;        /* longest tile list */
    uint64_t max_overlap;     /* largest depth overlap of volumes of interest in a tile */
    uint64_t max_active;      /* largest active set used by the tracer */
    uint64_t wide_tiles;      /* tiles traced on the wide-capacity path */
    uint64_t learned_accepted, learned_rejected;   /* relaxed steps (OVERRELAX, LEARNED) */
    uint64_t abuffer_binned;  /* tested candidates whose volume of interest a
                                 pixel ray of the tile meets (entries before
                                 the tile-level pruning) */
    uint64_t abuffer_candidates; /* (primitive, tile) pairs whose pixel
                                 rectangle touches the tile */
    uint64_t candidate_pixels[3]; /* pixels of the tested candidates' pixel
                                 rectangles inside their tiles (the per-ray
                                 test's work), by primitive kind: sphere, box,
                                 capsule */
    uint64_t abuffer_tested;  /* candidates left for the per-ray test: those
                                 alive for their tile's whole candidate set */
    uint64_t stalled;         /* blocks that stopped at their iteration bound
                                 before every ray finished (0 in a correct run) */
    uint64_t smooth_evals;    /* compact operators evaluated on their smooth
                                 (blending) branch */
    uint64_t block_cycles_max; /* longest 8x8 block of the trace, in shader
                                 clock cycles (s_memtime): the launch lasts
                                 at least this long */
    uint64_t block_cycles_sum; /* sum over the blocks (mean = sum / blocks) */
} st_stats;

/* Device memory allocator used for the scene's buffers (e.g. a framework's
 * caching allocator).  NULL allocator = hipMalloc / hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} st_allocator;

typedef struct st_scene st_scene;

/* Summary of a flattened scene (host struct). */
typedef struct {
    int32_t n_nodes, n_prims, depth;
    float extent;          /* largest edge of the primitives' bounding box */
    float lipschitz;       /* proven Lipschitz bound of the whole tree */
    float voi_lo[3], voi_hi[3];  /* bounding box of all volumes of interest */
    uint64_t device_bytes; /* device memory held by the scene (without A-buffer) */
    uint64_t abuffer_bytes;
} st_scene_info;

const char *st_status_str(st_status s);
const char *st_last_error(void);

/* Fill *t with the default tuning. */
st_status st_default_tuning(st_tuning *t);

/*
 * st_flatten_blobtree -- preprocessing of a blobtree (Section 4 storage and
 * Section 5 range-of-interest propagation; the paper runs it on the CPU only
 * when the tree structure changes).
 *   nodes[n] (host): the tree, root index `root`; n = 2P-1 for P primitives.
 *   alloc: allocator for the scene's device buffers (NULL: hipMalloc).
 *   stream: stream for the upload and the volume-of-interest kernel.
 *   *out: new scene handle, owned by the caller, freed by st_scene_destroy.
 * Work: validation, post-order relabelling, node bitfields, ranges of
 * interest (root (-inf,0]; a compact operator gives its children
 * max(d_o, d_parent), a sharp one d_parent), per-node Lipschitz factors,
 * pruning tables, then one host-to-device copy and a device pass computing
 * every primitive's volume of interest.
 * Errors: ST_E_TREE (not a binary tree over all n nodes, cycles, unknown
 * kind, depth > 31), ST_E_INVALID (NULL pointers, NaN/inf, radius/extent/k
 * <= 0, zero quaternion, 6 d_o - k <= 0), ST_E_NOMEM, ST_E_DEVICE.
 */
st_status st_flatten_blobtree(const st_node *nodes, int32_t n, int32_t root,
                              const st_allocator *alloc, void *stream, st_scene **out);

void st_scene_destroy(st_scene *s);

st_status st_scene_get_info(const st_scene *s, st_scene_info *info);

/*
 * st_update_primitives -- new parameters for existing primitives without
 * re-flattening (the paper's point that editing primitive parameters needs
 * no preprocessing, Sections 1 and 5: ranges of interest and Lipschitz
 * factors depend on the operators only).
 *   ids[n] (host): caller node indices of primitives; nodes[n] (host): their
 *   new values (same kind, left = right = -1, parameters validated as in
 *   st_flatten_blobtree).
 * Uploads the parameter blocks, recomputes every volume of interest on the
 * device and the scene's extent and box on the host, and marks the A-buffer
 * stale (st_trace returns ST_E_STALE until st_build_abuffer).  Synchronizes
 * `stream`.  Nothing is changed if any entry is rejected.
 * Errors: ST_E_INVALID (bad index, not a primitive, kind changed, invalid
 * parameters), ST_E_TREE (children given), ST_E_DEVICE.
 */
st_status st_update_primitives(st_scene *s, const int32_t *ids, const st_node *nodes, int32_t n, void *stream);

/*
 * st_build_abuffer -- per-tile A-buffer of volumes of interest (Section 6.2):
 * for every screen tile, the list of primitives whose volume of interest meets
 * a pixel-centre ray of the tile, with the tile's entry/exit view depth
 * (minimum entry, maximum exit over its rays), sorted by entry depth (ties by
 * primitive).  Built on the device by project (each primitive's pixel
 * rectangle; unless keep_all_entries, its candidate tiles cut to the screen
 * rectangles of the subtree boxes on the other side of its killing
 * ancestors) -> count per tile -> scan -> scatter candidates -> pruning of
 * each tile's candidate set -> per-tile ray test -> tile-level pruning of the
 * hits -> per-tile sort; the three cuts (see keep_all_entries) leave every
 * tile with the entries of the primitives that survive the dead-primitive
 * rule for its hits.  Synchronizes `stream` twice to size the A-buffer.  A build with the same camera and tuning as the scene's valid
 * A-buffer reruns every kernel with the sizes of the last build and does not
 * synchronize (the sizes are a function of scene, camera and tuning).
 *   cam (host), t (host, NULL = defaults).  The A-buffer is kept in the scene
 *   and tagged with the camera and tuning; st_trace refuses a different one.
 * Errors: ST_E_INVALID (camera size <= 0, fov outside (0,180), degenerate
 * basis, tile not 8/16/32), ST_E_NOMEM, ST_E_DEVICE.
 */
st_status st_build_abuffer(st_scene *s, const st_camera *cam, const st_tuning *t, void *stream);

/*
 * st_trace -- synchronized tracing (Algorithm 2): one wavefront per 8x8 pixel
 * block walks its tile's A-buffer list, segments the frustum into subfrustums
 * with a fixed active primitive set, builds the pruned tree of that set, and
 * sphere-traces every ray's span in it (Algorithm 3 evaluation).
 *   out_depth (device, float[H*W], row-major, row 0 top): t of the first
 *     surface crossing along the unit ray, +INFINITY on a miss;
 *   out_normal (device, float[H*W*3]): unit outward grad f/|grad f| at the
 *     hit, 0 on a miss;
 *   out_stats (host, may be NULL): counters; non-NULL makes the call
 *     synchronize `stream`.
 * Errors: ST_E_STALE (no A-buffer, or built for another camera), ST_E_INVALID,
 * ST_E_DEVICE.  Overlaps beyond max_active never fail (wide path).
 */
st_status st_trace(st_scene *s, const st_camera *cam, float *out_depth, float *out_normal,
                   st_stats *out_stats, void *stream);

/*
 * st_trace_ex -- st_trace with a per-pixel record (the paper's heat maps of
 * field evaluations per ray, Figure 1 and the Temple figure).
 *   out_info (device, uint32[H*W], may be NULL):
 *     bits 0-15  field evaluations of the ray (saturating),
 *     bit 16     hit, bit 17 stopped by max_steps (unconverged),
 *     bit 18     crossing refined by bracketing,
 *     bits 20-31 subfrustums the ray was traced in (saturating).
 * Other arguments, ownership and errors as st_trace.
 */
st_status st_trace_ex(st_scene *s, const st_camera *cam, float *out_depth, float *out_normal,
                      uint32_t *out_info, st_stats *out_stats, void *stream);

/*
 * st_trace_noalloc -- st_trace that allocates no device memory, for callers
 * that cannot allocate (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same kernels and the same outputs as
 * st_trace; the trace's scratch (one 208-byte counter record per 8x8 pixel
 * block, and the wide path's per-workgroup slots when an overlap is too large
 * for LDS) lives in a 32 MiB device array of the library, one copy per GPU,
 * held until the process ends.
 *   Arguments, layout and ownership as st_trace.  out_stats non-NULL makes
 *   the call synchronize `stream` (the counters are summed into the scene's
 *   own device words, allocated by st_flatten_blobtree).
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on the same GPU (two streams, two threads) race and give undefined
 * results; calls on one stream are ordered and safe.  The array needs no
 * clearing: every block writes its whole record.
 * Errors: ST_E_CAPACITY when the frame has more than 161,319 blocks of 8x8
 * pixels (about 11 million pixels; the message gives the sizes), or no room
 * is left for one wide-path slot; ST_E_STALE, ST_E_INVALID, ST_E_DEVICE as
 * st_trace.  Nothing is launched on a capacity error.
 */
st_status st_trace_noalloc(st_scene *s, const st_camera *cam, float *out_depth, float *out_normal,
                           st_stats *out_stats, void *stream);

/* Ancestor pointers of the ablation variants (Table 1 of the paper):
 * Algorithm 1 climbing parent pointers, or fast ancestor pointers. */
enum { ST_ABLATION_PARENT_PTR = 0, ST_ABLATION_FAST_PTR = 1 };

/*
 * st_trace_ablation -- the paper's ablation variants ParentPtr/Full and
 * FastPtr/Full (Table 1; Section 11, analysis of the rendering times): the
 * same images without synchronization.  A full-resolution dexel buffer is
 * built from the scene's A-buffer (for every pixel, the primitives whose
 * volume of interest its ray meets, with the ray's own entry and exit t,
 * sorted by address), then every ray is traced on its own: in each interval
 * of its list with a fixed active set it sphere-traces with the field
 * evaluated at every step by the sparse bottom-up traversal of Algorithm 1
 * (Section 7), climbing parent pointers (variant ST_ABLATION_PARENT_PTR) or
 * fast ancestor pointers (ST_ABLATION_FAST_PTR).  Stepping, refinement and
 * normals follow the A-buffer's tuning as in st_trace.
 *   Outputs and their layout as st_trace.  The dexel buffer is owned by the
 *   scene (grown on demand).  Synchronizes `stream` once to size it, and
 *   again when out_stats is non-NULL (abuffer_entries then counts the
 *   dexel entries, view_nodes the operators the traversals visited).
 * Errors: ST_E_STALE (no A-buffer for this camera), ST_E_INVALID (NULL
 * argument, unknown variant), ST_E_NOMEM, ST_E_DEVICE.
 */
st_status st_trace_ablation(st_scene *s, const st_camera *cam, int32_t variant, float *out_depth,
                            float *out_normal, st_stats *out_stats, void *stream);

/*
 * st_autotune -- picks, for this scene and camera, the tuning with the
 * shortest A-buffer build + trace time among a grid of A-buffer tile sizes
 * {8, 16, 32}, fetch caps max_new {6, 16, 64, 256} (the paper's 6 first) and
 * fetch-ahead depths sub_depth {1/20, 1/4} (the paper's 1/20 first).  Every
 * candidate is timed on the device with HIP events (median of `reps` runs,
 * reps >= 1) into temporary output buffers; the A-buffer is left built with
 * the winner, so st_trace can follow directly.
 *   base (host, NULL = defaults): fields other than the three searched ones.
 *   out (host): the chosen tuning; out_ms (host, may be NULL): its time.
 * Synchronous.  Errors: as st_build_abuffer and st_trace, ST_E_NOMEM.
 */
st_status st_autotune(st_scene *s, const st_camera *cam, const st_tuning *base, int32_t reps,
                      st_tuning *out, float *out_ms, void *stream);

/*
 * Step model (not in the paper; proposes omega for ST_STEP_LEARNED): an MLP
 * 8 -> 32 -> 32 -> 1 with ReLU and omega = 1 + 3 sigmoid(z), in [1, 4].
 * Parameters (ST_MLP_PARAMS floats, FP32 master copy): W1[32][8], b1[32],
 * W2[32][32], b2[32], w3[32], b3.  Features of a ray at a step (8 floats): the
 * plain step f/L, f/f_prev, the previous step, log2(1 + step index), the secant
 * slope of f along the ray divided by L, log2(1 + active primitives), t, and
 * log2(1 + pruned-view length); the model standardises them with norm[16] =
 * means[8], inverse standard deviations[8], and clamps them to [-3, 3].  Arithmetic: binary16 inputs,
 * weights and hidden activations, FP32 accumulation (matrix cores).
 * All array arguments of the st_mlp_* calls are device memory owned by the
 * caller; the calls are asynchronous on `stream`.
 */
#define ST_MLP_PARAMS 1377
#define ST_MLP_FEATURES 8
#define ST_MLP_TABLE_WORDS (59 * 64 + 16)

/* Pack weights and norm into the per-lane operand table of the inference
 * (uint32[ST_MLP_TABLE_WORDS]).  Errors: ST_E_INVALID (NULL), ST_E_DEVICE. */
st_status st_mlp_pack(const float *weights, const float *norm, uint32_t *table, void *stream);

/* omega[n] of raw features x[n][8] with a packed table, by the same device
 * function the tracer calls.  Errors: ST_E_INVALID (NULL with n > 0, n < 0),
 * ST_E_DEVICE. */
st_status st_mlp_forward(const uint32_t *table, const float *x, int32_t n, float *omega, void *stream);

/* Loss sum_i w_i (omega_i - target_i)^2 / n with w_i = over_weight (> 0)
 * where omega_i > target_i (an over-long proposal costs a rejected
 * evaluation), else 1, and its gradient with respect to weights (the binary16
 * roundings of the forward pass are passed through).  grad[ST_MLP_PARAMS] and
 * loss[1] are overwritten.  Errors: ST_E_INVALID, ST_E_DEVICE. */
st_status st_mlp_grad(const float *weights, const float *norm, const float *x, const float *target, int32_t n,
                      float over_weight, float *grad, float *loss, void *stream);

/* One Adam update of w[n] with moments m[n], v[n] (updated in place), bias
 * corrections for update number step >= 1.  Errors: ST_E_INVALID, ST_E_DEVICE. */
st_status st_mlp_adam(float *w, float *m, float *v, const float *grad, int32_t n, int32_t step, float lr,
                      float beta1, float beta2, float eps, void *stream);

/* Trains the step model on dumped samples (st_trace_dump) entirely on the
 * device: the feature standardisation (mean and 1 / max(std, 1e-6) per
 * feature, FP64 sums) into norm[16], initial weights from seed (He normal
 * hidden layers, small output layer, omega near 1.5 at the start), one
 * seeded order of the samples, then `epochs` passes of Adam (lr, betas 0.9 /
 * 0.999, eps 1e-8) over the full batches of `batch` samples, on the loss and
 * gradient of st_mlp_grad (the weight-gradient sums on the matrix cores).
 *   x (device float[n][8]) raw features, target (device float[n]) omega*;
 *   weights (device float[ST_MLP_PARAMS]) and norm (device float[16]) are
 *   outputs; losses (host float[epochs], may be NULL) gets each epoch's mean
 *   batch loss.  Blocks until done; allocates and frees its temporaries.
 * Not in the paper (the learned step is this library's addition).
 * Errors: ST_E_INVALID (NULL, n < 1 or > 2^31 - 1, epochs or batch < 1,
 * lr or over_weight <= 0), ST_E_NOMEM, ST_E_DEVICE. */
st_status st_train_step_model(const float *x, const float *target, int64_t n, int32_t epochs, int32_t batch,
                              float lr, float over_weight, uint64_t seed, float *weights, float *norm,
                              float *losses, void *stream);

/* Install a step model in the scene (weights and norm: device; packed into a
 * table the scene owns).  Required before tracing with ST_STEP_LEARNED.
 * Errors: ST_E_INVALID, ST_E_NOMEM, ST_E_DEVICE. */
st_status st_set_step_model(st_scene *s, const float *weights, const float *norm, void *stream);

/*
 * st_trace_dump -- training samples from the plain tracer: traces like
 * st_trace in ST_STEP_PLAIN whatever the tuning's step mode (same outputs),
 * and at each step where a relaxed step would be proposed (plain step >= eps
 * and ending before the subfrustum end) writes the ray's 8 features and the
 * target omega*: the largest omega in {1, 1.25, ..., 4} whose step (clamped
 * at the subfrustum end) passes the sphere-overlap test (1 if none).
 *   features (device, float[cap][8]), targets (device, float[cap]);
 *   *n_samples (host): samples produced; only the first min(n, cap) slots
 *   are written; their order is unspecified.  Synchronous.
 * Errors: as st_trace.
 */
st_status st_trace_dump(st_scene *s, const st_camera *cam, float *out_depth, float *out_normal,
                        float *features, float *targets, int64_t cap, int64_t *n_samples, void *stream);

/*
 * Batched rendering (not in the paper): many scenes, each with its camera,
 * rendered per frame by one graph launch.  A frame is: every scene's A-buffer
 * build replayed with the sizes of its first build (no host synchronization,
 * no allocation), then two persistent kernels pulling (scene, tile, 8x8
 * block) jobs from global atomic queues, longest tile list first (tiles within
 * the LDS capacity, then the wider ones).  Outputs are bitwise those of
 * st_trace on each scene with the same tuning.
 */
typedef struct st_batch st_batch;

/*
 * st_batch_create -- builds every scene's A-buffer once (sizing; synchronizes
 * `stream`), orders the jobs, and captures one frame into a HIP graph.
 *   scenes[n] (distinct handles; they must outlive the batch, and rebuilding
 *   one of their A-buffers elsewhere makes the batch stale), cams[n] (host),
 *   tuning (host, NULL = defaults; step mode must be ST_STEP_PLAIN),
 *   depths[n], normals[n]: device output buffers of each scene (as st_trace),
 *   fixed for the life of the batch.
 * Errors: ST_E_INVALID (NULL, n <= 0, repeated scene, non-plain step mode),
 * those of st_build_abuffer, ST_E_NOMEM, ST_E_DEVICE.
 */
st_status st_batch_create(st_scene *const *scenes, const st_camera *cams, int32_t n, const st_tuning *tuning,
                          float *const *depths, float *const *normals, void *stream, st_batch **out);

/* One frame: use_graph != 0 launches the captured graph on `stream`, 0
 * enqueues the same kernels directly.  Asynchronous.  Errors: ST_E_STALE (a
 * scene's A-buffer was rebuilt since creation), ST_E_DEVICE. */
st_status st_batch_render(st_batch *b, int32_t use_graph, void *stream);

/* Counters of the last frame, one st_stats per scene (out[cap], cap >= n).
 * Synchronizes `stream`. */
st_status st_batch_stats(const st_batch *b, st_stats *out, int32_t cap, void *stream);

void st_batch_destroy(st_batch *b);

/* Picks the batch tuning with the shortest graph frame among the grid of
 * st_autotune (tile {8,16,32}, max_new {6,16,64,256}, sub_depth {1/20, 1/4}),
 * timing `reps` replays of each candidate with HIP events (median).  Renders
 * into depths/normals; leaves the scenes' A-buffers built with the last
 * candidate.  Synchronous.  Errors: those of st_batch_create/render. */
st_status st_batch_autotune(st_scene *const *scenes, const st_camera *cams, int32_t n, const st_tuning *base,
                            float *const *depths, float *const *normals, int32_t reps, st_tuning *out,
                            float *out_ms, void *stream);

/* One-shot: create with default tuning, render once through the graph,
 * optional stats (stats[n], host), destroy.  Synchronous. */
st_status st_trace_batch(st_scene *const *scenes, const st_camera *cams, int32_t n, float *const *depths,
                         float *const *normals, st_stats *stats, void *stream);

/* Test hook: D (float[32][32], row-major) = A (float[32][8]) . B (float[8][32])
 * rounded to binary16 and multiplied by one matrix instruction, with D read
 * back through the accumulator layout the inference assumes.  Device arrays.
 * Errors: ST_E_INVALID, ST_E_DEVICE. */
st_status st_debug_mfma_probe(const float *A, const float *B, float *D, void *stream);

/*
 * st_debug_eval_field -- test hook: evaluates the pruned field f_A of a given
 * active primitive set at points (pruning semantics of Sections 7-9).  The
 * view is built by the same device code the tracer uses.
 *   active (host, caller's node indices of primitives, any order, no
 *     duplicates) or NULL for all primitives; n_active entries.
 *   pts (device, float[n_pts*3]); out_f (device, float[n_pts]);
 *   out_grad (device, float[n_pts*3], may be NULL).
 *   *out_root_used (host, may be NULL): 0 when the pruned root is unused
 *     (f_A is then +INFINITY everywhere: no surface in the volume).
 *   out_view (host, int32[view_cap], may be NULL): the device-built view as
 *     caller node indices in evaluation order; *out_view_len its length.
 * Synchronous.  Errors: ST_E_INVALID (bad index, duplicate, non-primitive),
 * ST_E_CAPACITY (active set beyond the library's largest view, 1024, or
 * view_cap too small), ST_E_DEVICE.
 */
st_status st_debug_eval_field(const st_scene *s, const int32_t *active, int32_t n_active,
                              const float *pts, int32_t n_pts, float *out_f, float *out_grad,
                              int32_t *out_root_used, int32_t *out_view, int32_t view_cap,
                              int32_t *out_view_len, void *stream);

/*
 * st_debug_prune_tree -- test hook, host only (no device needed): flattens
 * nodes[n] (same rules as st_flatten_blobtree) and builds the pruned tree view
 * of the active primitives with the same code the device runs after its LCA
 * step.  Writes the view in evaluation (post) order as caller node indices to
 * out_nodes[cap] and its length to *out_len (0 when the root is unused);
 * *out_lip gets the view's Lipschitz bound (may be NULL).
 * Errors: those of st_flatten_blobtree, ST_E_INVALID (bad active index),
 * ST_E_CAPACITY (cap too small).
 */
st_status st_debug_prune_tree(const st_node *nodes, int32_t n, int32_t root, const int32_t *active,
                              int32_t n_active, int32_t *out_nodes, int32_t cap, int32_t *out_len,
                              float *out_lip);

/*
 * st_debug_sparse_traversal -- test hook, host only (no device needed):
 * flattens nodes[n] (same rules as st_flatten_blobtree) and runs the sparse
 * bottom-up traversal of Algorithm 1 (Section 7: shadowing condition, stacked
 * operands popped at operators with two active operands; with fast pointers
 * the clamping to the stacked ancestor and the second pop condition) over the
 * active primitives, with the ignoreMod rules of Section 9 at operators
 * reached by one operand.  The same traversal code evaluates the field in
 * st_trace_ablation; here it is evaluated symbolically.  Writes the resulting
 * pruned expression in evaluation (post) order as caller node indices to
 * out_nodes[cap] (length *out_len, 0 when the root is unused), its Lipschitz
 * bound to *out_lip and the number of operators the traversal visited to
 * *out_visited (both may be NULL).
 *   variant: ST_ABLATION_PARENT_PTR or ST_ABLATION_FAST_PTR.
 * Errors: those of st_flatten_blobtree, ST_E_INVALID (bad active index or
 * variant), ST_E_CAPACITY (cap too small, or a traversal that did not end
 * with one value).
 */
st_status st_debug_sparse_traversal(const st_node *nodes, int32_t n, int32_t root, const int32_t *active,
                                    int32_t n_active, int32_t variant, int32_t *out_nodes, int32_t cap,
                                    int32_t *out_len, float *out_lip, int32_t *out_visited);

/*
 * st_debug_kernel_timing -- measurement hook: enable = 1 starts recording the
 *   duration of every launch of the binning's tile-test kernel on the build
 *   stream (a HIP event pair per launch, recorded on that stream; any earlier
 *   recording is discarded); enable = 0 stops, waits for the recorded events
 *   and returns the summed milliseconds and the number of launches.  The
 *   event pairs are created at the first recorded launches and kept by the
 *   scene.  Errors: ST_E_INVALID (NULL scene or outputs), ST_E_DEVICE.
 */
st_status st_debug_kernel_timing(st_scene *s, int32_t enable, float *total_ms, int32_t *launches);

/*
 * st_debug_abuffer -- test hook: copies the current A-buffer, as the tracer
 *   reads it (the entries kept by the tile-level pruning, each tile's list
 *   sorted by entry depth), to host memory: tile_off (host,
 *   uint32[n_tiles+1], offsets of the packed lists), entries (host, 3 x uint32
 *   per entry: caller node index of the primitive, z_in bits, z_out bits),
 *   capacities in elements; *n_tiles and *n_entries receive the sizes.  Pass
 *   NULL arrays to query sizes.  Synchronous.
 */
st_status st_debug_abuffer(const st_scene *s, uint32_t *tile_off, size_t tile_cap,
                           uint32_t *entries, size_t entry_cap, int32_t *n_tiles,
                           int64_t *n_entries, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ST_H */
