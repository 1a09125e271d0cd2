/*
 * nedf.h -- C ABI of the MI355X (gfx950) NeDF composition library.
 *
 * The library renders depth/ID buffers of many rigidly transformed neural
 * objects as in Gao et al., "A General Implicit Framework for Fast NeRF
 * Composition and Rendering" (AAAI 2024, arXiv 2308.04669):
 *   - nedf_march_depth     plain volume-rendered depth (Eq. 5) + Alg. 1 step 1
 *   - nedf_infer_depth_id  NeDF depth (Eq. 1, 2, 7) + Alg. 1 step 1, marcher
 *                          fallback for uncertain rays, secant refinement
 *   - nedf_shade_deferred  deferred shading (Eq. 8, Alg. 1 step 2)
 *   - nedf_shadow          shadow step (Alg. 2) and final composite
 *   - nedf_train_step      one forward/backward/Adam step of an intersection
 *                          network (Eq. 6 in regression form)
 *
 * Conventions for every entry point
 *   Ownership   Array arguments are DEVICE pointers owned by the caller unless
 *               the comment says "host".  The library never frees caller
 *               memory and never allocates device memory inside a call.
 *   Workspace   Calls that need scratch take (void* ws, size_t ws_bytes), a
 *               device buffer sized by nedf_workspace_size() for the same
 *               arguments.  Its first 256 bytes hold a device status word
 *               (read by nedf_check_status).
 *   Streams     Work is enqueued on `stream` (a hipStream_t; NULL = the
 *               default stream) and the call returns without synchronising.
 *               Host-side argument validation happens before anything is
 *               enqueued; a call that returns an error enqueued nothing.
 *   Errors      Every call returns an nedf_status; nedf_last_error() gives a
 *               thread-local message for the last failing call.
 *   Layout      Rays, points and directions are float32 [n][3] row-major;
 *               image buffers are row-major with pixel p = row * width + col,
 *               row 0 at the top.
 *   Alignment   Device pointers must be 16-byte aligned (NEDF_ERR_ALIGN).
 *   Concurrency Calls are reentrant; calls that share a workspace buffer
 *               must be ordered on one stream.
 */
#ifndef NEDF_H
#define NEDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* nedf_stream_t; /* hipStream_t */

typedef enum nedf_status {
  NEDF_OK = 0,
  NEDF_ERR_NULL = 1,        /* required pointer is NULL */
  NEDF_ERR_SHAPE = 2,       /* bad size, count or network shape */
  NEDF_ERR_DTYPE = 3,       /* unknown or unsupported precision */
  NEDF_ERR_ALIGN = 4,       /* device pointer not 16-byte aligned */
  NEDF_ERR_WORKSPACE = 5,   /* workspace smaller than nedf_workspace_size() */
  NEDF_ERR_CAPACITY = 6,    /* a device-side list overflowed (nedf_check_status) */
  NEDF_ERR_HIP = 7,         /* HIP runtime error */
  NEDF_ERR_UNSUPPORTED = 8  /* option combination not implemented */
} nedf_status;

typedef enum nedf_dtype {
  NEDF_F32 = 0,   /* float32 matrix cores (v_mfma_f32_32x32x2_f32) */
  NEDF_BF16 = 1,  /* bfloat16 inputs, float32 accumulate */
  NEDF_FP8 = 2,   /* OCP E4M3FN inputs with per-layer scales, float32 accumulate */
  NEDF_FP8_MX = 3 /* OCP MX: E4M3FN inputs with one power-of-two (E8M0) scale per 32 values along the
                     reduction, float32 accumulate; weight scales packed per output row, activation
                     scales formed in the kernel per sample (the smallest power of two that
                     brings the block's largest magnitude to at most 448).  Intersection network
                     (regression form) only; needs no calibration. */
} nedf_dtype;

/* Density field families of an object (local/canonical space). */
typedef enum nedf_field {
  NEDF_FIELD_SPHERE = 0,  /* sigma_max * sigmoid((radius - |x|) / width); param = {sigma_max, radius, width} */
  NEDF_FIELD_SLAB = 1,    /* sigma0 where z0 <= z <= z1; param = {sigma0, z0, z1} */
  NEDF_FIELD_MLP = 2      /* density network on gamma_L(x), see nedf_sigma_mode */
} nedf_field;

typedef enum nedf_sigma_mode {
  NEDF_SIGMA_SOFTPLUS = 0,         /* sigma = softplus(u) */
  NEDF_SIGMA_SOFTPLUS_MASKED = 1,  /* softplus(u), zero outside |x| <= bound */
  NEDF_SIGMA_SDF = 2               /* sigma_max * sigmoid(u - sdf_shape(x) / width);
                                      param = {sigma_max, width, shape} */
} nedf_sigma_mode;

typedef enum nedf_input_kind {
  NEDF_IN_XYZ = 0,       /* gamma_L(x), 3 (1 + 2L) features (density / NeRF trunk) */
  NEDF_IN_PLUECKER = 1,  /* gamma_L(d, o x d), 6 (1 + 2L) features (intersection network) */
  NEDF_IN_POINTS16 = 2   /* intersection network in the multi-level classifier form (Sec. "Intersection
                            network", Eq. 3-4, appendix architecture): gamma_L of 16 points on the line,
                            l ((2k + 1) / 16 - 1) from the tangency point along d, divided by l
                            (16 x 3 (1 + 2L) features); ReLU head to `width`, n_hidden residual blocks
                            h + ReLU(W2 ReLU(W1 h + b1) + b2), linear tail of n_out = 193 rows: hit
                            logit, 64 coarse and 128 fine bin logits.  Instantiated: L = 10, width 256,
                            16 blocks, F32 and BF16. */
} nedf_input_kind;

/*
 * Shape of a ReLU multilayer perceptron:
 *   in (encoded) -> n_hidden x [Linear(width) + ReLU] -> Linear(n_out)
 * and, when rgb_width > 0, a colour branch
 *   concat(h_last, gamma_dirL(d)) -> Linear(rgb_width) + ReLU -> Linear(3) -> sigmoid.
 * The packer accepts width in {64, 256}, n_hidden 1..16, n_out 1..2 and
 * rgb_width in {0, 128}; the kernels are instantiated for these shapes only
 * (other packed shapes are rejected with NEDF_ERR_UNSUPPORTED by the calls):
 *   density / NeRF trunk (xyz): width 64, 3 hidden, L6; width 256, 8 hidden,
 *     L10 (with the colour branch rgb_width 128, dir_L 4 for shading);
 *   intersection network (Pluecker): width 256, 8 hidden, L8 (F32, BF16, FP8);
 *   classifier form (NEDF_IN_POINTS16): width 256, L10, 1..64 residual
 *     blocks, n_out 193 (F32, BF16; training 1..16 blocks).
 */
typedef struct nedf_mlp_shape {
  int32_t in_kind;    /* nedf_input_kind */
  int32_t enc_L;      /* encoding levels of the input */
  int32_t width;
  int32_t n_hidden;
  int32_t n_out;
  int32_t rgb_width;  /* 0 = no colour branch */
  int32_t dir_L;      /* direction encoding levels of the colour branch */
} nedf_mlp_shape;

/* A packed network: a device blob written by nedf_pack_mlp (after upload). */
typedef struct nedf_mlp {
  nedf_mlp_shape shape;
  int32_t dtype;       /* nedf_dtype the blob was packed for */
  const void* blob;    /* device */
} nedf_mlp;

/* One object model: its density field in local space (marcher, fallback,
 * refinement, shading density), optional NeRF colour branch (inside the
 * density network), and optional intersection network F_Phi. */
typedef struct nedf_object {
  int32_t field;       /* nedf_field */
  int32_t sigma_mode;  /* nedf_sigma_mode (NEDF_FIELD_MLP) */
  float bound;         /* local bounding-sphere radius l (> 0) */
  float param[6];      /* field parameters, see nedf_field / nedf_sigma_mode */
  nedf_mlp density;    /* NEDF_FIELD_MLP: density network (blob may carry the colour branch) */
  nedf_mlp nedf;       /* intersection network (blob NULL when absent); in_kind PLUECKER, n_out 2 */
} nedf_object;

/* Instances of objects.  Rigid map G(q) = s R q + T (Eq. 7). */
typedef struct nedf_scene {
  int32_t n_objects;
  const nedf_object* objects;  /* host array of n_objects (at most NEDF_MAX_OBJECTS) */
  int32_t n_inst;
  const int32_t* inst_object;  /* device [n_inst]: object index of each instance */
  const float* inst_w2l;       /* device [n_inst][16]: world->local records from nedf_compose_transforms */
} nedf_scene;

#define NEDF_MAX_OBJECTS 32
#define NEDF_W2L_FLOATS 16

/* Rays: generated from a pinhole camera in-kernel, or explicit arrays. */
typedef struct nedf_camera {
  double eye[3], at[3], up[3];
  double fov_y_deg;        /* vertical field of view */
  int32_t width, height;   /* pixel centres; unit directions */
} nedf_camera;

typedef struct nedf_rays {
  int32_t kind;            /* 0 = camera, 1 = explicit arrays */
  nedf_camera camera;      /* kind 0: n = width * height */
  const float* origins;    /* kind 1: device [n][3] */
  const float* dirs;       /* kind 1: device [n][3], unit length */
  int64_t n;               /* kind 1: number of rays */
} nedf_rays;

typedef struct nedf_march_opts {
  int32_t n_samples;       /* midpoint samples per (ray, instance) pair, 1..4096 */
  int32_t clip_to_bound;   /* 1: march the chord of the local bounding sphere;
                              0: march the fixed world interval [t_near, t_far] */
  float t_near, t_far;
  float hit_threshold;     /* hit iff opacity >= hit_threshold (default 0.5) */
  int32_t dtype;           /* precision of MLP fields */
} nedf_march_opts;

/* Options of the NeDF path (Eq. 1, 2, 7 with marcher fallback and refinement). */
typedef struct nedf_infer_opts {
  int32_t dtype;            /* precision of fallback/refinement density fields; the intersection
                               networks run in their blob's dtype (this dtype, NEDF_FP8 or
                               NEDF_FP8_MX) */
  float p_lo, p_hi;         /* hit probability band sent to the marcher (inclusive), default 0.2 / 0.8 */
  int32_t refine_steps;     /* secant updates on the winning pixel (0 = off), default 3 */
  float refine_h;           /* seed offset in the object's own units (world offset refine_h * s for an
                               instance of scale s), default 0.05 */
  nedf_march_opts march;    /* marcher used for fallback pairs (clip_to_bound must be 1) */
} nedf_infer_opts;

/* Options of deferred shading (Eq. 8, Alg. 1 step 2). */
typedef struct nedf_shade_opts {
  int32_t K;                /* samples per pixel in [D - h, D + h]: 1, 2, 4, 8, 16 or 32 (K = 1 is Eq. 8) */
  float h;                  /* half width in world units, default 0.05 */
  float clear_rgb[3];       /* colour of pixels without an ID */
  int32_t dtype;
  float rs_sigma;           /* outlier threshold (Sec. "Deferred Shading"): a pixel whose density is below
                               it at every one of its K samples did not reach the surface and is shaded
                               again by volume rendering over the bounding chord; 0 = off */
  int32_t rs_samples;       /* samples over the chord for those pixels: 8, 16 or 32 */
} nedf_shade_opts;

/* Options of the shadow step (Alg. 2). */
typedef struct nedf_shadow_opts {
  float eps;                /* depth bias epsilon (world units) */
  float beta;               /* attenuation 0 < beta < 1 per shadowing light */
  int32_t method;           /* 0 = NeDF path (nedf_infer_opts), 1 = plain marcher */
  nedf_infer_opts infer;    /* depth method of the shadow rays */
  uint32_t directional_mask;  /* bit m set: light m is directional (lights[m] is its direction of travel,
                                 normalised by the library); otherwise a point light at lights[m] */
  float dir_distance;       /* directional lights: shadow rays start this far from x against the light
                               direction (must exceed the distance from any hit point to the farthest
                               bounding sphere along that direction) */
} nedf_shadow_opts;

/* ---------------------------------------------------------------- helpers */
const char* nedf_version(void);
const char* nedf_last_error(void);
const char* nedf_status_string(int32_t status);

/*
 * Bytes of the packed blob of a network (nedf_pack_mlp).  0 when the shape
 * or dtype is unsupported (nedf_last_error says why).
 */
size_t nedf_mlp_packed_bytes(const nedf_mlp_shape* shape, int32_t dtype);

/*
 * Pack float32 weights into the blob layout the GPU kernels read (matrix-core
 * fragment order, per-lane bias and head tables).  HOST only: W[i]/b[i] are
 * HOST pointers to layer i in PyTorch layout [out][in] / [out], layers in
 * order (hidden layers, head, then colour-branch hidden and colour head; for
 * NEDF_IN_POINTS16: head, the two layers of each residual block, tail).
 * `out` is a HOST buffer of nedf_mlp_packed_bytes() bytes; the caller uploads
 * it to the device.  For NEDF_FP8, `fp8_scales` (host, 2 per hidden layer:
 * weight scale, activation scale) is required; otherwise it is ignored.
 */
int32_t nedf_pack_mlp(const nedf_mlp_shape* shape, int32_t dtype, const float* const* W,
                      const float* const* b, const float* fp8_scales, void* out, size_t out_bytes);

/*
 * World->local records of the instances (Sec. "Manipulating Objects", Eq. 7),
 * composed in float64 on the GPU and rounded to float32:
 *   in  inst_G   device float64 [n][13] = R (row-major 3x3), T (3), s
 *   out inst_w2l device float32 [n][16] = R^T (9), -R^T T / s (3), s, 1/s, 0, 0
 * so that o_l = R^T o / s + c and d_l = R^T d.
 */
int32_t nedf_compose_transforms(const double* inst_G, int32_t n, float* inst_w2l,
                                nedf_stream_t stream);

typedef enum nedf_op {
  NEDF_OP_MARCH = 0,
  NEDF_OP_INFER = 1,
  NEDF_OP_SHADE = 2,
  NEDF_OP_SHADOW = 3
} nedf_op;

/* Workspace bytes needed by an entry point for these arguments. */
/* pair_capacity <= 0 sizes the (ray, instance) pair list for the worst case
 * n_rays * n_inst; a smaller explicit capacity is reported as NEDF_ERR_CAPACITY
 * by nedf_check_status when exceeded (results are then incomplete). */
size_t nedf_workspace_size(int32_t op, const nedf_scene* scene, const nedf_rays* rays,
                           int64_t pair_capacity);

/*
 * Synchronise `stream` and return the device status word of `ws`
 * (NEDF_OK, or NEDF_ERR_CAPACITY when a pair list overflowed).
 */
int32_t nedf_check_status(const void* ws, nedf_stream_t stream);

/*
 * Stage timing.  nedf_profile_enable(1) clears the record list and makes every
 * later call bracket its kernel launches with HIP events on its stream, under
 * stage names ("depth.cull", "march.mlp", ...; a stage run inside another is
 * named "outer/inner", e.g. "shadow/infer.nedf"); nedf_profile_enable(0) stops
 * recording.  nedf_profile_read synchronises on the recorded events and
 * returns, per stage in first-seen order, the summed elapsed milliseconds and
 * the number of brackets: names is a host buffer of max_stages x 64 chars.
 */
int32_t nedf_profile_enable(int32_t on);
int32_t nedf_profile_read(int32_t max_stages, char* names, double* total_ms, int32_t* counts,
                          int32_t* n_stages);

/*
 * Counters of the last call that used `ws` (synchronises `stream`):
 * [0] (ray, instance) pairs after culling (or binned pixels of
 * the last per-pixel stage), [1] work items of that list, [2] pairs decided
 * by the intersection network, [3] pairs sent to the marcher, [4] pairs the
 * network classified as misses, [5] marcher pairs left after the depth test
 * against the network's hits (a pair entering its bounding sphere beyond the
 * pixel's nearest hit cannot change the result and is not marched), [6]
 * (ray, instance) pairs after the last culling.  Host int64 out[7].
 */
int32_t nedf_ws_counters(const void* ws, nedf_stream_t stream, int64_t* out7);

/* ------------------------------------------------------------- hot path */

/*
 * Plain volume-rendering marcher (Eq. 5) composed over all instances
 * (Alg. 1 step 1).  For every (ray, instance) pair whose ray meets the
 * instance's bounding sphere (or every pair, clip_to_bound = 0), the local
 * ray is marched with N midpoint samples, giving opacity A = sum w_i and
 * depth D = s * sum w_i t_i / A.  The pair hits when A >= hit_threshold.
 *   depth    [n] float32: minimum hit depth over instances, +inf if none
 *   id       [n] int32: instance of that minimum (lowest index on ties), -1 if none
 *   opacity  [n] float32 or NULL: max over instances of A
 */
int32_t nedf_march_depth(const nedf_scene* scene, const nedf_rays* rays,
                         const nedf_march_opts* opts, float* depth, int32_t* id,
                         float* opacity, void* ws, size_t ws_bytes, nedf_stream_t stream);

/*
 * NeDF depth and ID buffers (Alg. 1 step 1 with Eq. 7): for every (ray,
 * instance) pair meeting the instance's bounding sphere, the object's
 * intersection network maps the local line (d, o x d) to (mu_hat, z);
 * D = s (t_perp - l clamp(mu_hat, -1, 1)), p = sigmoid(z).  p > p_hi is a hit
 * at D (if D > 0), p < p_lo a miss; the band [p_lo, p_hi] and origins inside
 * the bounding sphere are resolved by the plain marcher of the object's
 * density field.  The minimum over instances gives depth/id (ties: lowest
 * index).  With refine_steps > 0 the winner's depth is refined by secant
 * steps on the surface function of its density field (SDF-mode networks and
 * spheres; others are left as is).
 * Every object must carry an intersection network (nedf.blob) or be an
 * analytic field (marched directly).
 *   depth [n] float32, id [n] int32 (-1 = none)
 */
int32_t nedf_infer_depth_id(const nedf_scene* scene, const nedf_rays* rays, const nedf_infer_opts* opts,
                            float* depth, int32_t* id, void* ws, size_t ws_bytes, nedf_stream_t stream);

/*
 * Buffer reuse while one object is manipulated (Sec. "CUDA implementation":
 * the other objects' rendering is frozen and their buffers reused).  The
 * depth of nedf_infer_depth_id is the minimum over instances of a per-pair
 * key; split the instances into disjoint sets, keep the keys of the sets that
 * do not move, recompute only the moving set's keys each frame, and merge.
 *
 * nedf_infer_keys: the first half of nedf_infer_depth_id (culling, the
 * intersection networks, the marcher fallback) on `scene`, typically a
 * subset of the full scene's instances, writing for every ray the key
 * (float bits of the world depth << 32) | instance, or 0x7F800000FFFFFFFF
 * (no hit), into keys [n] (device, uint64, 16-byte aligned, written whole).
 * inst_gid (device int32 [scene->n_inst], or NULL for the identity) gives the
 * index each instance of `scene` has in the full scene; that index is what
 * the key carries, and what breaks ties.  The refinement options are not
 * used here.  ws as for nedf_infer_depth_id on `scene`; the pair-list status
 * is read with nedf_check_status(ws).
 *
 * nedf_compose_keys: merges 1..8 key buffers (device uint64 [n] each, the
 * key_sets array itself on the host) by their per-ray minimum and finishes
 * as nedf_infer_depth_id does (depth/id, then secant refinement on the full
 * `scene`, which must hold every instance the keys name).  For disjoint sets
 * covering the full scene, and the same rays and options, depth and id are
 * bit-identical to one nedf_infer_depth_id call on the full scene.  A key
 * naming an instance >= scene->n_inst is dropped and sets NEDF_ERR_SHAPE in
 * the status word of ws (nedf_check_status).  ws: the refinement bins at
 * most one pair per ray, so nedf_workspace_size(NEDF_OP_INFER, scene, rays,
 * n) bytes suffice.
 */
int32_t nedf_infer_keys(const nedf_scene* scene, const nedf_rays* rays, const nedf_infer_opts* opts,
                        const int32_t* inst_gid, uint64_t* keys, void* ws, size_t ws_bytes,
                        nedf_stream_t stream);
int32_t nedf_compose_keys(const nedf_scene* scene, const nedf_rays* rays, const nedf_infer_opts* opts,
                          const uint64_t* const* key_sets, int32_t n_sets, float* depth, int32_t* id,
                          void* ws, size_t ws_bytes, nedf_stream_t stream);

/*
 * nedf_infer_depth_id for callers that cannot allocate device memory (code
 * under HIP graph capture, fixed-memory serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, with the workspace taken
 * from a fixed device array of nedf_static_scratch_bytes() (64 MiB) that
 * every GPU the library runs on holds until the process ends.  The caller
 * still passes inputs and outputs.  A call whose worst case, every ray
 * meeting every instance (nedf_workspace_size(NEDF_OP_INFER, scene, rays, 0)
 * bytes), exceeds the array is rejected with NEDF_ERR_WORKSPACE before any
 * work, so no pair list can overflow.  Calls no hipMalloc or hipFree and
 * records no profiling events.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (several streams or host threads)
 * race; calls in sequence on a stream do not (each clears what it uses).
 */
int32_t nedf_infer_depth_id_static(const nedf_scene* scene, const nedf_rays* rays,
                                   const nedf_infer_opts* opts, float* depth, int32_t* id,
                                   nedf_stream_t stream);
size_t nedf_static_scratch_bytes(void);

/*
 * Deferred shading (Eq. 8, Alg. 1 step 2): every pixel with a valid id is
 * shaded by its object's NeRF colour branch at K samples around its depth,
 * composited locally (K = 1 is the single evaluation of Eq. 8); pixels
 * without an id get clear_rgb; analytic objects use param[3..5] as colour.
 *   depth [n], id [n] inputs; rgb [n][3] float32 output
 */
int32_t nedf_shade_deferred(const nedf_scene* scene, const nedf_rays* rays, const float* depth,
                            const int32_t* id, const nedf_shade_opts* opts, float* rgb, void* ws,
                            size_t ws_bytes, nedf_stream_t stream);

/*
 * Shadow step (Alg. 2) for n_lights point or directional lights (host float32
 * [n_lights][3], at most 8; directional_mask in the options): for each pixel
 * with a valid id, x = o + D d; a ray from each light towards x (for a
 * directional light with direction l: from x - dir_distance l along l, an
 * orthographic shadow ray) is resolved like step 1 over all instances (depth D_L);
 * D_L + eps < |L - x| (directional: < dir_distance) multiplies the pixel's
 * factor by beta.
 *   shadow [n] float32 output multiplier; rgb_inout [n][3] (nullable) is
 *   multiplied by it (final composite: colour buffer x shadow buffer).
 */
int32_t nedf_shadow(const nedf_scene* scene, const nedf_rays* rays, const float* depth, const int32_t* id,
                    const float* lights, int32_t n_lights, const nedf_shadow_opts* opts, float* shadow,
                    float* rgb_inout, void* ws, size_t ws_bytes, nedf_stream_t stream);

/* ------------------------------------------------------------- training */

/* Adam and loss settings of nedf_train_step (Eq. 6 regression form, or the
 * classifier form for NEDF_IN_POINTS16 networks; the paper trains with Adam
 * at lr 5e-4). */
typedef struct nedf_train_opts {
  float lr, beta1, beta2, eps;  /* Adam (Kingma & Ba 2015), bias-corrected */
  float w_hit;                  /* weight of the hit BCE term (0.1 in Eq. 6) */
  float bound;                  /* local bounding radius l: mu* = (t_perp - D) / l */
} nedf_train_opts;

/* Bytes of the device training state of a network (float32 master weights,
 * Adam moments, last-step gradients, bfloat16 weight copies, step counter).
 * The network must have width 256 and n_out = 2 (regression form) or be a
 * classifier-form network (NEDF_IN_POINTS16, L10, 1..16 blocks). */
size_t nedf_train_state_bytes(const nedf_mlp_shape* shape);

/* Device workspace bytes of nedf_train_step for a batch of B rays. */
size_t nedf_train_workspace_size(const nedf_mlp_shape* shape, int32_t B);

/* Initialise a state from float32 DEVICE weights W[i] [out][in] / b[i]
 * (hidden layers, then the head); moments, gradients and step become zero. */
int32_t nedf_train_init(const nedf_mlp_shape* shape, const float* const* W, const float* const* b,
                        void* state, size_t state_bytes, nedf_stream_t stream);

/*
 * One training step on B local rays (B a multiple of 256): forward pass in
 * bfloat16 on the matrix cores with float32 accumulation, loss
 *   L = (1/B) sum_i [alpha_i (mu_hat_i - mu*_i)^2 + w_hit BCEwithLogits(z_i, alpha_i)]
 * with mu* = (t_perp - depth_label) / bound and alpha = hit_label (Eq. 6,
 * regression form, labels from the inverse of Eq. 2), back-propagation and
 * one Adam update of the float32 master weights.
 *   o_l, d_l     device float32 [B][3] local rays (d unit)
 *   depth_label  device float32 [B] local depth of the first surface
 *   hit_label    device uint8 [B]
 *   loss_out     device float32 [3]: total, masked MSE, BCE (before the update)
 * A classifier-form network (NEDF_IN_POINTS16: head, 2 layers per residual
 * block, 1..16 blocks, tail of 193 rows) trains on Eq. 6 itself: target bins
 * (c, f) = S(mu*) (u = (mu* + 1) / 2, c = floor(64 u), f = floor(128 (64 u - c)),
 * clamped), L = (1/B) sum_i [alpha_i (mean_j BCE(v_c,ij, [j = c_i]) +
 * mean_j BCE(v_f,ij, [j = f_i])) + w_hit BCE(alpha_hat_i, alpha_i)], and
 * loss_out = total, bin term, hit term.
 */
int32_t nedf_train_step(const nedf_mlp_shape* shape, void* state, const float* o_l, const float* d_l,
                        const float* depth_label, const uint8_t* hit_label, int32_t B,
                        const nedf_train_opts* opts, float* loss_out, void* ws, size_t ws_bytes,
                        nedf_stream_t stream);

/* Copy the float32 master weights (which = 0) or the last step's gradients
 * (which = 1) of a state into DEVICE arrays W[i] [out][in] / b[i]. */
int32_t nedf_train_export(const nedf_mlp_shape* shape, const void* state, int32_t which, float* const* W,
                          float* const* b, nedf_stream_t stream);

/* ------------------------------------------------------------- FP8 */

/* Device workspace bytes of nedf_fp8_calibrate for a batch of B rays. */
size_t nedf_fp8_calibrate_workspace_size(const nedf_mlp_shape* shape, int32_t B);

/*
 * Per-layer E4M3 scales of a network (width 256, n_out 2): a bfloat16 forward
 * pass over B calibration rays (o_l, d_l device float32 [B][3], B a multiple
 * of 256) records the largest |activation| entering every hidden layer; the
 * weight scale is the largest |weight| of that layer.  scales (device float32
 * [2 n_hidden]) receives {w_scale, a_scale} = amax / 448 per hidden layer,
 * the layout nedf_pack_mlp expects for NEDF_FP8 (after a copy to the host).
 * W[i] / b[i] are DEVICE float32 layers as for nedf_train_init.
 */
int32_t nedf_fp8_calibrate(const nedf_mlp_shape* shape, const float* const* W, const float* const* b,
                           const float* o_l, const float* d_l, int32_t B, float* scales, void* ws,
                           size_t ws_bytes, nedf_stream_t stream);

/*
 * Autotuning.  Not a step of the paper's method: a tuning aid for the grouped
 * launches that evaluate every (ray, instance) pair of Alg. 1 per object.
 * The tunable launch shape of the matrix-core kernels is encoded as
 * 1000 * (waves / 4 - 1) + 100 * (blocks - 1) + 10 * occupancy + superchunk:
 * the waves of a workgroup (4 or 8; eight waves share one copy of each weight
 * chunk in LDS), the number of 32-row blocks each wave carries through the
 * network (1 or 2; two blocks share every weight read from LDS), the number
 * of persistent workgroups per CU (1 or 2) and the number of 32-row weight
 * chunks streamed into LDS per copy and barrier (1, 2 or 4).  NEDF_TUNE_SLABS is the number of depth slabs in
 * which nedf_infer_depth_id runs the intersection network front to back
 * (1, 2, 4, 8, 16 or 32; an exact pruning: a pair whose smallest possible
 * depth lies beyond the pixel's nearest hit is skipped).  It is kept per
 * kernel and dtype in a process-wide
 * table guarded by a mutex (the library's only global state besides the
 * profiler).
 *
 * nedf_tune_candidates writes the values instantiated for (kernel, dtype) into
 * out (up to NEDF_TUNE_MAX) and their number into n.  nedf_tune_get/nedf_tune_set read and
 * write the table (set rejects values that are not candidates with
 * NEDF_ERR_UNSUPPORTED).  nedf_autotune runs the stage of `kernel` on the
 * caller's inputs once per candidate (`reps` timed runs each, after one
 * warm-up), keeps the fastest in the table and describes the trial in
 * *report (host).  `opts` is a nedf_march_opts* for NEDF_TUNE_MARCH (plain
 * marcher, nedf_march_depth) and a nedf_infer_opts* for NEDF_TUNE_NEDF and
 * NEDF_TUNE_SLABS (nedf_infer_depth_id, tuning the intersection-network
 * kernel of `dtype`);
 * depth and id are caller-owned device outputs of n_rays elements; ws as for
 * those calls.  Synchronises `stream`.
 */
typedef enum { NEDF_TUNE_MARCH = 0, NEDF_TUNE_NEDF = 1, NEDF_TUNE_SLABS = 2 } nedf_tune_kernel;
#define NEDF_TUNE_MAX 8

typedef struct {
  int32_t kernel, dtype;
  int32_t n_candidates;
  int32_t candidate[NEDF_TUNE_MAX];
  float ms[NEDF_TUNE_MAX];
  int32_t chosen;
} nedf_tune_report;

int32_t nedf_tune_candidates(int32_t kernel, int32_t dtype, int32_t* out, int32_t* n);
int32_t nedf_tune_get(int32_t kernel, int32_t dtype, int32_t* value);
int32_t nedf_tune_set(int32_t kernel, int32_t dtype, int32_t value);
int32_t nedf_autotune(int32_t kernel, int32_t dtype, const nedf_scene* scene, const nedf_rays* rays,
                      const void* opts, float* depth, int32_t* id, void* ws, size_t ws_bytes, int32_t reps,
                      nedf_stream_t stream, nedf_tune_report* report);

#ifdef __cplusplus
}
#endif
#endif /* NEDF_H */
