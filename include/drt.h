/*
 * drt.h -- C ABI of the MI355X differentiable path tracer.
 *
 * The library implements the data-parallel hot path of Path Replay
 * Backpropagation as described in the Dr.Jit paper (Jakob, Speierer, Roussel,
 * Vicini, "Dr.Jit: A Just-In-Time Compiler for Differentiable Rendering",
 * ACM TOG 41(4), 2022):
 *   - a primal path-tracing megakernel (megakernel #1 of Fig. "prb-structure",
 *     Sec. "Physically Based Differentiable Rendering"),
 *   - a replayed adjoint megakernel that regenerates every sample, recovers
 *     the incident radiance at each vertex by subtraction ("arithmetic
 *     invertibility"), and scatter-adds parameter gradients with atomics
 *     (megakernels #2 and #3 of the same figure, fused; Sec. "Differentiating
 *     polymorphism" on implicit reads becoming atomic scatter-reductions;
 *     Sec. "AD tape surgery" on detached sampling),
 *   - the image loss and the optimiser step around them.
 *
 * Conventions
 *   - Every function returns a drt_status and never throws.  On failure the
 *     thread-local message drt_last_error() says why.
 *   - Argument errors return DRT_EINVAL before anything is enqueued.
 *   - GPU work is enqueued asynchronously on `hip_stream` (a hipStream_t, or
 *     NULL for the default stream); errors inside kernels surface at the next
 *     synchronisation.  A launch failure returns DRT_EHIP.
 *   - "device" pointers are HIP device memory owned by the caller (PyTorch
 *     tensors in the Python binding); they must stay valid until the stream
 *     work that uses them has completed.  "host" pointers are read during the
 *     call only.
 *   - Images are float32 [n_cams][height][width][3], row 0 at the top.
 *     Textures are float32 [height][width][3].
 */
#ifndef DRT_H
#define DRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DRT_OK = 0,
  DRT_EINVAL = -1,      /* invalid argument (nothing was enqueued) */
  DRT_ENOMEM = -2,      /* host allocation failed */
  DRT_EHIP = -3,        /* a HIP call or kernel launch failed */
  DRT_ESTATE = -4,      /* object in the wrong state */
  DRT_EUNSUPPORTED = -5 /* valid request beyond the library's limits */
} drt_status;

/* Message of the last failure on the calling thread ("" if none). */
const char* drt_last_error(void);

/* Library version string. */
const char* drt_version(void);

enum { DRT_MAX_TEXTURES = 8, DRT_MAX_CAMERAS = 32 };

/* BSDF types of the material switch (the paper's polymorphic BSDF call,
 * Sec. "Running example", dispatched here by a switch on this id). */
enum {
  DRT_BSDF_NULL = 0,             /* pass-through, counts as a vertex, skipped by shadow rays */
  DRT_BSDF_DIFFUSE = 1,          /* Lambertian rho/pi (albedo constant or textured) */
  DRT_BSDF_DIFFUSE_TEXTURED = 2, /* Lambertian with a texture (texture >= 0 required) */
  DRT_BSDF_CONDUCTOR = 3,        /* GGX microfacet reflection, Schlick Fresnel with f0 */
  DRT_BSDF_DIELECTRIC = 4,       /* rough GGX dielectric, exact Fresnel, index eta */
  DRT_BSDF_PLASTIC = 5,          /* GGX coat (index eta) over a Lambertian base */
  DRT_BSDF_TWOSIDED = 6,         /* Lambertian on both sides */
  DRT_BSDF_MASK = 7              /* Lambertian with stochastic opacity, else pass-through */
};

/* Emitter types. */
enum {
  DRT_EMITTER_AREA = 0,        /* one-sided quad p0 + u e1 + v e2, front = e1 x e2 */
  DRT_EMITTER_ENV = 1,         /* latitude-longitude environment map of the scene */
  DRT_EMITTER_DIRECTIONAL = 2  /* p0 = unit direction towards the light, radiance = irradiance */
};

/* Render flags. */
enum {
  DRT_FLAG_NO_NEE = 1,          /* BSDF sampling only (no next-event estimation, no MIS) */
  DRT_FLAG_CACHE_INPUT_GRAD = 2, /* drt_render_adjoint_cached: differentiate the cache's
                                    output through its albedo and roughness inputs too */
  DRT_FLAG_GLOBAL_SCENE = 4      /* read the tree and triangles from device memory even where
                                    the scene fits the megakernels' per-workgroup LDS copy
                                    (same results; for comparisons) */
};

typedef struct {
  int32_t type;          /* DRT_BSDF_* */
  int32_t texture;       /* albedo texture index, or -1 for the constant albedo */
  int32_t rough_slot;    /* index into the roughness parameter array, or -1 for alpha */
  int32_t reserved;
  float albedo[3];       /* constant albedo */
  float alpha;           /* constant GGX roughness (not squared) */
  float f0[3];           /* conductor reflectance at normal incidence */
  float eta;             /* dielectric / plastic index of refraction */
  float opacity;         /* mask opacity in [0, 1] */
  float reserved2[3];
} drt_material;

typedef struct {
  int32_t type;          /* DRT_EMITTER_* */
  int32_t reserved[3];
  float p0[3], e1[3], e2[3];
  float radiance[3];
} drt_emitter;

typedef struct {
  int32_t width, height;
} drt_texture_desc;

/* Scene description: host arrays, read during drt_scene_plan/upload only. */
typedef struct {
  int32_t n_vertices, n_triangles;
  const float* positions;        /* [n_vertices][3] */
  const float* uvs;              /* [n_vertices][2], or NULL (all zero) */
  const int32_t* indices;        /* [n_triangles][3]; winding gives the geometric normal */
  const int32_t* tri_material;   /* [n_triangles] */
  const int32_t* tri_emitter;    /* [n_triangles], -1 if the triangle does not emit */
  int32_t n_materials;
  const drt_material* materials;
  int32_t n_emitters;
  const drt_emitter* emitters;
  int32_t n_textures;            /* <= DRT_MAX_TEXTURES */
  const drt_texture_desc* textures;
  int32_t n_roughness;           /* length of the roughness parameter array */
  const float* envmap;           /* [env_height][env_width][3], or NULL */
  int32_t env_width, env_height;
} drt_scene_desc;

typedef struct drt_scene drt_scene; /* opaque, library-owned host object */

typedef struct {
  int32_t n_nodes, n_leaves, max_depth, forced_leaves;
  int32_t n_triangles, n_materials, n_emitters, n_textures, n_roughness;
  int32_t env_width, env_height;
  float eps;                     /* ray-spawn offset: 1e-4 x largest extent of the scene box */
  float bounds_lo[3], bounds_hi[3];
  uint64_t device_bytes;         /* bytes of the scene's device buffer actually used */
  int32_t lds_copy;              /* 1: the rendering megakernels read the tree, triangles,
                                    shading records, materials and emitters from a copy in
                                    each workgroup's LDS (the scene fits 5 KB and its tree
                                    at most 5 four-wide levels); 0: from device memory */
} drt_scene_info;

/* Upper bound of the device bytes a scene needs (no BVH build). */
drt_status drt_scene_plan(const drt_scene_desc* desc, uint64_t* device_bytes);

/* Build the scene on the host -- binned-SAH BVH flattened to 64-byte
 * two-child nodes and 48-byte triangle records, material/emitter tables
 * (the paper's closure-data array, appendix "Dynamic dispatch to closures"),
 * environment sampling tables -- and copy it into the caller's device buffer
 * (>= drt_scene_plan bytes, 256-byte aligned).  Blocks until the copy is done.
 * The device buffer must outlive the scene object. */
drt_status drt_scene_upload(const drt_scene_desc* desc, void* device_buffer, uint64_t buffer_bytes,
                            void* hip_stream, drt_scene** out);

/* Same build, written into a HOST buffer instead (for inspection/caching). */
drt_status drt_scene_pack(const drt_scene_desc* desc, void* host_buffer, uint64_t buffer_bytes,
                          drt_scene** out);

drt_status drt_scene_info_get(const drt_scene* scene, drt_scene_info* out);
drt_status drt_scene_destroy(drt_scene* scene);

typedef struct {
  float origin[3], target[3], up[3];
  float fov_y_deg;               /* vertical field of view */
  int32_t width, height;         /* all cameras of one call share width and height */
} drt_camera;

/* Differentiable parameters (device, caller-owned). */
typedef struct {
  const float* textures[DRT_MAX_TEXTURES]; /* [H][W][3] each, per scene texture */
  const float* roughness;                  /* [n_roughness], or NULL if n_roughness == 0 */
} drt_params;

/* Gradient outputs (device, caller-owned).  The adjoint ADDS into them; the
 * caller zeroes them.  A NULL entry skips that parameter. */
typedef struct {
  float* textures[DRT_MAX_TEXTURES];
  float* roughness;
} drt_grads;

typedef struct {
  int32_t spp;        /* samples per pixel, >= 1; n_cams*W*H*spp <= 2^46, else
                         DRT_EUNSUPPORTED */
  int32_t max_depth;  /* D: path segments including the camera ray, 1..65536 */
  int32_t rr_depth;   /* Russian roulette after sampling at vertex k >= rr_depth */
  uint32_t flags;     /* DRT_FLAG_* */
  uint64_t seed;      /* Philox key */
  uint64_t* stats;    /* device uint64[DRT_STAT_COUNT] accumulators, or NULL (see DRT_STAT_*) */
} drt_render_opts;

/* Indices into drt_render_opts.stats. */
enum {
  DRT_STAT_RAYS = 0,      /* closest-hit rays traced */
  DRT_STAT_SHADOW = 1,    /* shadow rays traced */
  DRT_STAT_NODES = 2,     /* BVH nodes visited */
  DRT_STAT_TRIS = 3,      /* ray/triangle tests */
  DRT_STAT_VERTICES = 4,  /* scattering vertices shaded */
  DRT_STAT_SCATTER = 5,   /* gradient atomics issued (adjoint) */
  DRT_STAT_LREM_MAX = 6,  /* adjoint: max over samples of |L_rem| / |L| at the path's end
                             (max norms over channels; |L_rem| itself where L = 0), as
                             float bits: the replay's relative residual */
  DRT_STAT_SAMPLES = 7,   /* samples traced */
  DRT_STAT_TEX_LANES = 8, /* adjoint: lanes that scatter-added a texel gradient */
  DRT_STAT_TEX_KEYS = 9,  /* adjoint: distinct texels among the lanes of each wave-wide
                             texel scatter, summed: TEX_LANES / TEX_KEYS is the mean
                             number of lanes per distinct texel (measurement only;
                             counting them costs a ballot loop per scatter) */
  /* SIMD utilisation by phase, counted by the stats kernels of
     drt_render_forward and drt_render_adjoint (0 elsewhere): each event
     once per wave, to set beside the per-lane count of the same event */
  DRT_STAT_WAVE_NODES = 10,  /* node-loop iterations of waves (per lane: NODES) */
  DRT_STAT_WAVE_TRIS = 11,   /* triangle-loop iterations of waves (per lane: TRIS) */
  DRT_STAT_LANE_STEPS = 12,  /* vertex steps of live paths, per lane */
  DRT_STAT_WAVE_STEPS = 13,  /* vertex steps of waves */
  DRT_STAT_WAVE_SHADE = 14,  /* shading blocks entered by waves (per lane: VERTICES) */
  DRT_STAT_COUNT = 15
};

/* Primal rendering (Fig. "prb-structure", megakernel #1): for each pixel
 * the mean of spp path-traced samples (box filter of one-pixel support).
 * Sample s of pixel (cam, x, y) draws Philox4x32-10 blocks with key = seed
 * and counter = (g_lo, g_hi, b, dim), g = ((cam*H + y)*W + x)*spp + s.
 * image: device float [n_cams][H][W][3], overwritten.  With spp >= 2 the
 * samples of a pixel are summed in two halves (by two workgroups) that are
 * added onto the zeroed image; the result is deterministic (two addends
 * onto zero commute exactly) but may differ in the last bit from one
 * running sum. */
drt_status drt_render_forward(const drt_scene* scene, const drt_params* params,
                              const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                              float* image, void* hip_stream);

/* Reverse-mode derivative of sum_p <adj_image_p, I_p> (megakernels #2 and
 * #3 fused): each sample is traced once to get its radiance L, then replayed
 * with the same random numbers, subtracting each vertex's emission and
 * next-event term from L to recover the radiance arriving over the sampled
 * direction; with detached sampling the gradient of a vertex is
 * dL . (d NEE_k + L_rem * (d f_k) / f_k).  opts->seed is the replay seed (use
 * a seed different from the primal's for a decorrelated gradient).
 * adj_image: device float [n_cams][H][W][3].  Gradients are added. */
drt_status drt_render_adjoint(const drt_scene* scene, const drt_params* params,
                              const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                              const float* adj_image, const drt_grads* grads, void* hip_stream);

/* drt_render_adjoint with intersection records: pass A keeps, per step of
 * each lane's current sample, its closest hit (triangle, barycentrics) and
 * its shadow ray's outcome in hit_records, and the replay reads them back
 * instead of tracing the same rays again (the replay's sampling, L_rem
 * subtraction and scatter are unchanged, so are the gradients, up to atomic
 * order).  The launch runs as many workgroups as the current device holds
 * at once; they take the work units (an 8x8 tile and one of min(spp, 4)
 * ranges of its samples) from a counter, and each keeps its records in its own
 * slot, reused sample after sample -- so the size depends on the device and
 * max_depth, not on spp and, past the device's size, not on the image:
 * drt_render_adjoint_hit_bytes(n_cams, W, H, spp, max_depth) = 256 B
 * (counter) + min(resident workgroups, work units) x max_depth x 64 lanes x
 * 16 B, for the current device (0 for invalid sizes).  hit_records: device
 * scratch of at least that many bytes, 16-byte aligned, overwritten; calls
 * that overlap on one buffer race. */
int64_t drt_render_adjoint_hit_bytes(int32_t n_cams, int32_t width, int32_t height, int32_t spp,
                                     int32_t max_depth);
drt_status drt_render_adjoint_hits(const drt_scene* scene, const drt_params* params,
                                   const drt_camera* cams, int32_t n_cams,
                                   const drt_render_opts* opts, const float* adj_image,
                                   const drt_grads* grads, void* hit_records, int64_t hit_bytes,
                                   void* hip_stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc:
 * drt_render_adjoint_hits with the intersection records and the work
 * counter in a scratch array that the library holds in device memory
 * instead of a caller buffer.  Same arguments, results and conventions
 * otherwise (gradients ADDED to grads).  The array holds
 * DRT_NOALLOC_SCRATCH_BYTES (256 B counter + 32 MiB of record slots); each
 * GPU the library runs this on keeps its own copy until the process ends.
 * Sizes whose drt_render_adjoint_hit_bytes() exceeds it return
 * DRT_EUNSUPPORTED before anything is enqueued (with 4096 resident
 * workgroups, as on MI355X: max_depth <= 8).  Calls nothing that allocates
 * (no hipMalloc / hipFree); the counter is cleared by a fill kernel on the
 * stream.  All calls on one GPU share its array: calls that overlap on one
 * GPU (on any streams) race. */
#define DRT_NOALLOC_SCRATCH_BYTES (256 + (32LL << 20))
drt_status drt_render_adjoint_noalloc(const drt_scene* scene, const drt_params* params,
                                      const drt_camera* cams, int32_t n_cams,
                                      const drt_render_opts* opts, const float* adj_image,
                                      const drt_grads* grads, void* hip_stream);

/* The primal image by the wavefront variant of the same estimator (same
 * sample streams and conventions as drt_render_forward): per bounce, a
 * closest-hit kernel, a shading kernel and a shadow-ray kernel exchange the
 * path state through the workspace (the execution model the paper's
 * megakernels are compared with, Sec. "Evaluation").  For the comparison;
 * opts->stats is ignored.  workspace: device scratch of at least
 * drt_render_wavefront_workspace_bytes(n_cams*W*H*spp) bytes, 16-byte
 * aligned (the size is 0 for n_paths < 0 or > 2^46, the largest sample
 * count of one rendering call). */
int64_t drt_render_wavefront_workspace_bytes(int64_t n_paths);
drt_status drt_render_wavefront(const drt_scene* scene, const drt_params* params,
                                const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                                void* workspace, int64_t workspace_bytes, float* image,
                                void* hip_stream);

/* The replayed adjoint by the wavefront variant: pass A (the primal with
 * opts->seed, radiance per path) and pass B (the replay with the
 * subtractions and the gradient scatter) as per-bounce kernels exchanging
 * the path state through the workspace.  Same gradients as
 * drt_render_adjoint (ADDED to grads) up to float rounding and atomic order.
 * workspace: at least drt_render_adjoint_wavefront_workspace_bytes(
 * n_cams*W*H*spp) bytes, 16-byte aligned (0 for n_paths < 0 or > 2^46). */
int64_t drt_render_adjoint_wavefront_workspace_bytes(int64_t n_paths);
drt_status drt_render_adjoint_wavefront(const drt_scene* scene, const drt_params* params,
                                        const drt_camera* cams, int32_t n_cams,
                                        const drt_render_opts* opts, const float* adj_image,
                                        const drt_grads* grads, void* workspace,
                                        int64_t workspace_bytes, void* hip_stream);

/* Checkpointed adjoint: the naive way to differentiate a path tracer that
 * Sec. "Evaluation" measures Path Replay Backpropagation against -- one
 * checkpoint per scattering event instead of a replay.
 * drt_render_checkpointed_forward renders the image (same estimator, sample
 * streams and arithmetic as drt_render_wavefront) and keeps, in the
 * workspace, the ray state of every path before every bounce (64 B per path
 * and bounce: memory grows with opts->max_depth).
 * drt_render_checkpointed_adjoint then walks the bounces backwards from those
 * checkpoints: it recomputes each vertex (closest hit, shading with
 * derivatives, shadow ray), forms its gradient with the radiance collected
 * by the later vertices, and adds the vertex's own terms to that radiance.
 * The gradient of sum <adj_image, image> is ADDED to grads; it equals
 * drt_render_adjoint's with the same seed up to float rounding and atomic
 * order.  Both calls take the same scene, params, cams and opts, and the
 * adjoint call needs the workspace as the forward call left it (no other
 * use in between).  workspace: at least
 * drt_render_checkpointed_workspace_bytes(n_cams*W*H*spp, opts->max_depth)
 * bytes, 16-byte aligned (the size function returns 0 for max_depth outside
 * [1, 65536] or n_paths outside [0, 2^40]). */
int64_t drt_render_checkpointed_workspace_bytes(int64_t n_paths, int32_t max_depth);
drt_status drt_render_checkpointed_forward(const drt_scene* scene, const drt_params* params,
                                           const drt_camera* cams, int32_t n_cams,
                                           const drt_render_opts* opts, void* workspace,
                                           int64_t workspace_bytes, float* image,
                                           void* hip_stream);
drt_status drt_render_checkpointed_adjoint(const drt_scene* scene, const drt_params* params,
                                           const drt_camera* cams, int32_t n_cams,
                                           const drt_render_opts* opts, const float* adj_image,
                                           const drt_grads* grads, void* workspace,
                                           int64_t workspace_bytes, void* hip_stream);

/* Forward-mode derivative of the primal image along a parameter direction
 * (Sec. "Physically Based Differentiable Rendering" describes the forward
 * mode used to check and visualise derivatives): image_tangent = d I / d params
 * . direction, [n_cams][H][W][3] float, written (not added).  The direction
 * uses the drt_grads layout, read only: direction->textures[t] [H][W][3] per
 * scene texture (NULL: zero), direction->roughness one value per slot (NULL:
 * zero).  Same sample streams, detached sampling and attached BSDF values
 * as drt_render_adjoint, so with equal opts <adj, image_tangent> equals
 * <gradient from drt_render_adjoint(adj), direction> up to rounding. */
drt_status drt_render_jvp(const drt_scene* scene, const drt_params* params, const drt_camera* cams,
                          int32_t n_cams, const drt_render_opts* opts, const drt_grads* direction,
                          float* image_tangent, void* hip_stream);

/* Ray queries against the scene BVH.
 * rays: device float [n][8] = (ox, oy, oz, tmin, dx, dy, dz, tmax), d unit length.
 * mode 0 (closest): hits[i] = {t, b1, b2, prim} with prim = -1 on a miss;
 *   ties in t go to the lowest triangle id.
 * mode 1 (any): prim = 1 if any non-null triangle is hit in (tmin, tmax), else -1. */
typedef struct {
  float t, b1, b2;
  int32_t prim;
} drt_hit;
drt_status drt_trace(const drt_scene* scene, const float* rays, int64_t n, int32_t mode,
                     drt_hit* hits, void* hip_stream);

/* Philox4x32-10: out[i] = philox(counter[i], key[i]).
 * counters: device uint32 [n][4]; keys: device uint32 [n][2]; out: device uint32 [n][4]. */
drt_status drt_philox(const uint32_t* counters, const uint32_t* keys, int64_t n, uint32_t* out,
                      void* hip_stream);

/* L2 image loss l = (1/n) sum (img - target)^2 and its adjoint
 * adj = 2 (img - target) / n (the image-space adjoint that drives the
 * adjoint pass).  img, target, adj: device float [n] (adj may be NULL: loss
 * only); loss: device float [1]; workspace: device float
 * [drt_loss_workspace_floats(n)] (per-block partial sums, overwritten).  The
 * sum is carried in float32 pairs (error-free two-sum and fma product
 * error), accurate to about 2^-44 before the final rounding to float. */
int64_t drt_loss_workspace_floats(int64_t n);
drt_status drt_loss_l2(const float* img, const float* target, int64_t n, float* adj, float* loss,
                       float* workspace, void* hip_stream);

/* Adam (Kingma & Ba) step t >= 1 with bias correction, then clamp to [lo, hi]:
 * param, m, v updated in place; grad read, and reset to zero afterwards if
 * zero_grad != 0 (ready for the next adjoint, which accumulates).
 * All device float [n]. */
typedef struct {
  float lr, beta1, beta2, eps;
  int32_t step;
  float lo, hi;
  int32_t zero_grad;
  uint16_t* half_out; /* device FP16 copy of the updated parameters, or NULL */
} drt_adam_opts;
drt_status drt_adam_step(float* param, float* grad, float* m, float* v, int64_t n,
                         const drt_adam_opts* opts, void* hip_stream);

/* ------------------------------------------------------------------------
 * Neural radiance cache.  The paper does not cover it; the library adds it as
 * a learned replacement of path tails: paths stop at their record vertex --
 * the first scattering vertex with index >= K, after that vertex's emission
 * -- and add beta * max(C, 0), where C is a small network evaluated on an
 * encoding of the vertex.  The network is trained online on records of plain
 * paths whose target is the radiance they collected after the record point,
 * divided by the throughput there.
 *
 * Record (float[16]): position[3], direction back along the ray[3], normal
 * facing that direction[3], roughness (1 unless microfacet), albedo[3]
 * (f0 for a conductor, 1 for a dielectric), then target[3] (training) or
 * throughput[3] (queries).
 * Encoding (80 inputs): 16-level hash grid of the position normalised to
 * bbox (2 FP16 features per entry, 2^log2_table entries per level,
 * resolutions base_res..max_res geometrically, trilinear; dense indexing while
 * (N+1)^3 entries fit, else the spatial hash of Mueller et al. 2022), 16 real
 * spherical harmonics (bands 0-3) of the direction and of the normal,
 * roughness, albedo, zero padding.
 * Network: 80 -> 64 -> 64 -> 64 -> 64 -> 3, ReLU, no biases; weights are one
 * float array [DRT_NRC_WEIGHTS] of row-major [out][in] matrices, rounded to
 * BF16 inside the kernels; BF16 MFMA with FP32 accumulation.
 * ------------------------------------------------------------------------ */
enum { DRT_NRC_INPUTS = 80, DRT_NRC_WEIGHTS = 17600, DRT_NRC_RECORD = 16, DRT_NRC_LEVELS = 16 };

typedef struct {
  int32_t levels;        /* must be 16 */
  int32_t features;      /* must be 2 */
  int32_t log2_table;    /* entries per level = 2^log2_table, 10..24 */
  int32_t base_res, max_res;
  int32_t trunc_vertex;  /* K >= 2 */
  float bbox_lo[3], bbox_hi[3];
} drt_nrc_config;

/* Encoding only (test hook): records [n][16] -> x [n][80] float. */
drt_status drt_nrc_encode(const drt_nrc_config* cfg, const uint16_t* grid, const float* records,
                          int64_t n, float* x, void* hip_stream);

/* Network only (test hooks): y [n][3] = net(x); inputs rounded to BF16.
 * backward: dW [DRT_NRC_WEIGHTS] += d<dy, y>/dW; dx [n][80] = d<dy, y>/dx for
 * inputs 0..31 (the hash features), 0 for the others; dx may be NULL.  The
 * backward runs the training kernels' backward and weight-gradient passes
 * and needs their workspace (drt_nrc_train_workspace_bytes(n), 16-byte
 * aligned). */
drt_status drt_nrc_forward(const float* weights, const float* x, int64_t n, float* y,
                           void* hip_stream);
drt_status drt_nrc_backward(const float* weights, const float* x, const float* dy, int64_t n,
                            void* workspace, int64_t workspace_bytes, float* dW, float* dx,
                            void* hip_stream);

/* Hash-grid gradient only (test hook): dgrid [levels][2^log2_table][2] +=
 * the trilinear scatter of dx [n][80] (inputs 0..31) at the records'
 * positions. */
drt_status drt_nrc_grid_backward(const drt_nrc_config* cfg, const float* records, const float* dx,
                                 int64_t n, float* dgrid, void* hip_stream);

/* Training paths: path j (Philox counter g = j, key opts->seed) starts at the
 * pixel floor(r n_pix / 2^32), r = first word of block (camera, dim 2), runs a
 * plain path (opts->max_depth, rr_depth, flags; spp is ignored) and writes
 * records[j] and valid[j]; *count = number of valid records (set, not added).
 * records: device float [n_paths][16]; valid: device int32 [n_paths]. */
drt_status drt_nrc_collect(const drt_scene* scene, const drt_params* params,
                           const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                           const drt_nrc_config* cfg, int64_t n_paths, float* records,
                           int32_t* valid, int32_t* count, void* hip_stream);

/* Bytes of device workspace drt_nrc_train needs for n records (the BF16
 * layer inputs and output gradients of every record, 1216 B per record
 * rounded up to 16-record tiles); 0 for n < 0 or n > 2^31, the range
 * drt_nrc_train accepts. */
int64_t drt_nrc_train_workspace_bytes(int64_t n);

/* One training pass: relative-L2 loss (Mueller et al. 2021: mean over valid
 * records and channels of (y - t)^2 / (y^2 + 0.01), y held fixed in the
 * denominator) -> network and grid gradients ADDED to dW [17600] and dgrid
 * [levels][2^log2_table][2] (float); *loss is set to the loss.  workspace:
 * device scratch of at least drt_nrc_train_workspace_bytes(n) bytes,
 * 16-byte aligned (overwritten). */
drt_status drt_nrc_train(const drt_nrc_config* cfg, const float* weights, const uint16_t* grid,
                         const float* records, const int32_t* valid, const int32_t* count,
                         int64_t n, void* workspace, int64_t workspace_bytes, float* dW,
                         float* dgrid, float* loss, void* hip_stream);

/* Self-training records of the radiance cache (the cache's answer closes
 * each training path, so the records see radiance beyond any fixed depth).
 * n_paths paths, path j starting at the pixel chosen as in drt_nrc_collect,
 * run the cached estimator with record vertex tail_vertex (first scattering
 * vertex with index >= tail_vertex, before opts->max_depth; opts->spp is
 * ignored): the radiance up to that vertex plus beta * max(C, 0) there, C
 * answered by the network (weights, grid as in drt_render_forward_cached).
 * Every scattering vertex k < tail_vertex on the way writes record
 * j * (tail_vertex - 1) + k - 1 of records [n_paths * (tail_vertex - 1)][16]:
 * features (as in drt_nrc_collect) and target = (path estimate - radiance
 * collected up to and including vertex k's emission) / beta_k per channel
 * (0 where beta_k is 0) -- the radiance scattered from vertex k.  valid
 * [n_paths * (tail_vertex - 1)]: 1 for the records written (others are
 * zeroed); *count = their number.  The result feeds drt_nrc_train with
 * n = n_paths * (tail_vertex - 1).  workspace: device scratch of at least
 * drt_nrc_collect_self_workspace_bytes(n_paths, tail_vertex) bytes.
 * 2 <= tail_vertex <= 32; n_paths <= INT32_MAX and
 * n_paths * (tail_vertex - 1) <= 2^31 (the size function returns 0 outside
 * 2 <= tail_vertex <= 32, 0 <= n_paths <= INT32_MAX).  The paper does not study caches; this
 * is the self-training of Mueller et al. (2021) written on the cached
 * estimator. */
int64_t drt_nrc_collect_self_workspace_bytes(int64_t n_paths, int32_t tail_vertex);
drt_status drt_nrc_collect_self(const drt_scene* scene, const drt_params* params,
                                const drt_camera* cams, int32_t n_cams,
                                const drt_render_opts* opts, const drt_nrc_config* cfg,
                                const float* weights, const uint16_t* grid, int32_t tail_vertex,
                                int64_t n_paths, float* records, int32_t* valid, int32_t* count,
                                void* workspace, int64_t workspace_bytes, void* hip_stream);

/* Device state of a radiance cache (all caller-owned device memory).  The
 * gradient buffers must be zero on the first frame; each frame leaves them
 * zero again. */
typedef struct {
  float* weights;          /* [DRT_NRC_WEIGHTS] FP32 master weights */
  float* weights_m;        /* [DRT_NRC_WEIGHTS] Adam first moments */
  float* weights_v;        /* [DRT_NRC_WEIGHTS] Adam second moments */
  float* weights_grad;     /* [DRT_NRC_WEIGHTS] gradient accumulator */
  float* grid;             /* [levels][2^log2_table][2] FP32 master features */
  float* grid_m, *grid_v;  /* same size: Adam moments */
  float* grid_grad;        /* same size: gradient accumulator */
  uint16_t* grid_half;     /* same size, FP16: the copy the kernels read; rewritten each frame */
  float* records;          /* [n_records][16], n_records = n_paths (plain records) or
                              n_paths (K - 1) (self-training with tail vertex K) */
  int32_t* valid;          /* [n_records] */
  int32_t* count;          /* [1] */
  void* train_workspace;   /* drt_nrc_train_workspace_bytes(n_records) bytes, 16-byte aligned */
  int64_t train_workspace_bytes;
  void* self_workspace;    /* self-training: drt_nrc_collect_self_workspace_bytes(n_paths, K) */
  int64_t self_workspace_bytes;
  float* loss;             /* [1]: the frame's training loss */
} drt_nrc_state;

typedef struct {
  int64_t n_paths;         /* training paths of the frame */
  int32_t self_training;   /* 0: records of plain paths at the truncation vertex
                              (drt_nrc_collect); K >= 2: self-training records of paths
                              closed by the cache at vertex K (drt_nrc_collect_self) */
  int32_t step;            /* Adam step t >= 1 of this frame */
  float lr, beta1, beta2, eps;
} drt_nrc_frame_opts;

/* One training frame of the radiance cache, enqueued on the stream:
 * records (drt_nrc_collect, or drt_nrc_collect_self with the current
 * network) -> one fused training pass (drt_nrc_train: relative-L2 loss,
 * network and hash-grid gradients) -> Adam on the weights and on the grid
 * (step frame->step; gradients re-zeroed; the FP16 grid rewritten).  opts
 * carries the training paths' seed, max_depth, rr_depth and flags (spp is
 * ignored).  All arguments are checked before anything is enqueued. */
drt_status drt_nrc_train_frame(const drt_scene* scene, const drt_params* params,
                               const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                               const drt_nrc_config* cfg, const drt_nrc_frame_opts* frame,
                               const drt_nrc_state* state, void* hip_stream);

/* Entries of the int32 query scratch of the cached calls for `capacity`
 * queries: ids [capacity] | order [capacity] | spatial keys [capacity] |
 * parameter references [capacity][2] | one padding entry if capacity is
 * odd | sort pairs [capacity][2] | bin histogram [32768]; 0 for
 * capacity < 0 or > 2^40, which the cached calls reject.  The scratch must
 * be 8-byte aligned (the calls reject it otherwise). */
int64_t drt_nrc_query_ints(int64_t capacity);

/* Primal render with the cache: image = (1/spp) sum over samples of the
 * path radiance up to the record vertex plus beta * max(C, 0) there.  The
 * queries are sorted by the Morton code of their position's cell among
 * 512^3 cells of the cache's box (by its 32^3 bin alone when capacity <
 * 2^20) before the network answers them (hash-table gathers of nearby
 * queries share cache lines).  Scratch (device, overwritten): queries float [capacity][16],
 * query_ints int32 [drt_nrc_query_ints(capacity)], query_count int32 [1];
 * capacity >= n_cams*W*H*spp <= INT32_MAX.  The cache terms are added with
 * float atomics (summation order not deterministic). */
drt_status drt_render_forward_cached(const drt_scene* scene, const drt_params* params,
                                     const drt_camera* cams, int32_t n_cams,
                                     const drt_render_opts* opts, const drt_nrc_config* cfg,
                                     const float* weights, const uint16_t* grid, float* queries,
                                     int32_t* query_ints, int32_t* query_count,
                                     int64_t capacity, float* image, void* hip_stream);

/* Reverse-mode gradient of the cached estimator.  The term beta * max(C, 0)
 * at the record vertex reaches earlier vertices' BSDF derivatives through
 * beta, as in the PRB replay of Sec. "Physically Based Differentiable
 * Rendering".  Without DRT_FLAG_CACHE_INPUT_GRAD in opts->flags that is all
 * (cache output detached).  With it, the network is differentiated as well,
 * through the inputs that are scene parameters: each query's output
 * gradient dL * beta * [C > 0] (dL = adj of its pixel / spp) is propagated
 * back through the network (BF16 operands, FP32 accumulation) to the albedo
 * and roughness inputs, which are added to the texel and roughness slot the
 * record vertex read them from (albedo of a conductor or dielectric and
 * roughness of a non-microfacet type are constants: nothing is added);
 * the network weights and the hash grid receive nothing.  Launches on the
 * stream: a cached pass with seed opts->seed that writes each sample's
 * truncated radiance to sample_radiance and its query (with the sample
 * index) to queries / query_ints; the network answers the queries into
 * sample_radiance; with the flag, one more network pass over the queries
 * adds the input term; the replay then starts every sample from its stored
 * estimate (no second forward pass).  Gradients are ADDED to grads as in
 * drt_render_adjoint.  sample_radiance: device float [n_cams*W*H*spp][3]
 * (scratch); queries, query_ints, query_count and capacity as for
 * drt_render_forward_cached.  hit_records (optional, null: the replay traces
 * its rays again): device scratch of at least
 * drt_render_adjoint_cached_hit_bytes(n_cams, W, H, spp, max_depth) bytes
 * (records for every sample: workgroups of 8x8 pixels x spp x max_depth x
 * 64 lanes x 16 B), 16-byte aligned; the cached pass writes them and the
 * replay reads them instead of tracing. */
int64_t drt_render_adjoint_cached_hit_bytes(int32_t n_cams, int32_t width, int32_t height,
                                            int32_t spp, int32_t max_depth);
drt_status drt_render_adjoint_cached(const drt_scene* scene, const drt_params* params,
                                     const drt_camera* cams, int32_t n_cams,
                                     const drt_render_opts* opts, const drt_nrc_config* cfg,
                                     const float* weights, const uint16_t* grid, float* queries,
                                     int32_t* query_ints, int32_t* query_count, int64_t capacity,
                                     float* sample_radiance, const float* adj_image,
                                     const drt_grads* grads, void* hit_records, int64_t hit_bytes,
                                     void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* DRT_H */
