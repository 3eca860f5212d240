/* meshrf -- hybrid surface-volumetric ray marcher for MI355X (gfx950).
 *
 * C ABI of the rendering path of "Dynamic Mesh-Aware Radiance Fields"
 * (Qiao, Gao et al., ICCV 2023): each ray marches a radiance field (hash grid +
 * small MLPs, linear HDR colour), alpha-composites radiance and throughput,
 * finds the closest mesh surface through a BVH and scatters off mirror, glass
 * or diffuse surfaces, with shadow rays to point lights, for any number of
 * bounces (Sec. 3.1 "Hybrid Rendering Algorithm", Algorithm 1, Eq. 8-13).
 *
 * Conventions (all entry points):
 *  - Every call returns an mr_status; on failure mr_last_error() returns a
 *    thread-local message.  Arguments are validated on the host before any
 *    launch; a call that fails validation touches no memory.
 *  - Pointers named host_* are host memory read during the call only.  All
 *    other array pointers are device memory owned by the caller; they must stay
 *    valid until the stream reaches the call.  Handles are owned by the library
 *    and released by the matching *_destroy.
 *  - stream is a hipStream_t passed as void*; NULL is the null stream.  Render
 *    calls are asynchronous on it and never synchronise with the host, so they
 *    can be captured into a HIP graph.
 *  - Arrays of 3-vectors are row-major (n, 3) float32.
 */
#ifndef MESHRF_H
#define MESHRF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MR_OK = 0,
  MR_ERR_INVALID_ARG = 1, /* bad shape, value or pointer                  */
  MR_ERR_OOM = 2,         /* device or host allocation failed             */
  MR_ERR_DEVICE = 3,      /* a HIP call failed                            */
  MR_ERR_UNSUPPORTED = 4, /* valid but not implemented (e.g. network size) */
  MR_ERR_STATE = 5        /* handle in the wrong state                    */
} mr_status;

/* Message of the last failed call on this thread ("" if none). */
const char* mr_last_error(void);

/* Library version string. */
const char* mr_version(void);

enum { MR_F32 = 0, MR_F16 = 1, MR_BF16 = 2 };
enum { MR_MIRROR = 0, MR_GLASS = 1, MR_DIFFUSE = 2 };
enum { MR_SAMPLER_UNIFORM = 0, MR_SAMPLER_PROPOSAL = 1 };

/* ------------------------------------------------------------------------ */
/* Radiance field: multiresolution hash grid + density MLP + colour MLP     */
/* (the pretrained Instant-NGP field of Sec. 3.3; colour in linear HDR as   */
/* required by Sec. 3.1 "Unifying color space").                            */
/*                                                                          */
/* Level l has integer resolution N_l.  Vertex v of level l is stored at    */
/* vx + vy(N+1) + vz(N+1)^2 when (N+1)^3 <= 2^log2_table_size, otherwise at */
/* (vx ^ vy*2654435761 ^ vz*805459861) mod 2^log2_table_size (uint32).      */
/* A point p maps to xhat = (p - aabb_min)/(aabb_max - aabb_min), clamped   */
/* to [0,1]; corners floor(xhat N) (at most N-1) + {0,1}^3, trilinear.      */
/* Features are level-major, zero padded to density_in.                     */
/* density: h = relu(W0 f), raw = W1 h (density_out values, no biases),     */
/*          sigma = softplus(raw[0] + density_offset).                      */
/* colour:  c_in = raw ++ SH(d) (real orthonormal SH, sh_components of      */
/*          1/4/9/16, Condon-Shortley phase), zero padded to color_in;      */
/*          color_hidden_layers ReLU layers of width color_hidden, then a   */
/*          3-wide output layer; rgb = exp(out).                            */
/* A proposal field has color_hidden_layers = 0 and density_out = 1.        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_levels;           /* 1..16 */
  int32_t feats_per_level;    /* 2 */
  int32_t log2_table_size;    /* 10..24 */
  const int32_t* host_resolutions; /* n_levels integers >= 1 */
  int32_t table_dtype;        /* MR_F32 or MR_F16 (device copy of the table) */
  int32_t mlp_dtype;          /* MR_F32, or MR_BF16 (MFMA with FP32 accumulation) */
  int32_t density_in, density_hidden, density_out;
  int32_t color_in, color_hidden, color_hidden_layers, sh_components;
  float density_offset;
  float aabb_min[3], aabb_max[3];
} mr_field_desc;

typedef struct mr_field mr_field;

/* Create a field from FP32 master parameters.
 * host_table: [n_levels][2^log2_table_size][feats_per_level] float32.
 * host_mlp:   all layers in forward order, each [out][in] row-major float32:
 *             density (hidden x density_in), (density_out x hidden), colour
 *             (color_hidden x color_in), (color_hidden x color_hidden) per
 *             extra hidden layer, (3 x color_hidden).  For a proposal field
 *             (color_hidden_layers = 0) only the two density layers.
 * Supported shapes: density_in = 32 (or n_levels*feats <= 16 for a proposal),
 * density_hidden = 64 (16 for a proposal), density_out = 16 (1), color_in =
 * 32, color_hidden = 64, and (n_levels, sh_components, color_hidden_layers)
 * one of (8, 4, 1), (16, 16, 2), (16, 4, 1), (8, 16, 2); a proposal field
 * has 5 levels.  Non-finite parameters are MR_ERR_INVALID_ARG; other shapes
 * are MR_ERR_UNSUPPORTED, refused before anything is allocated.  The table
 * is converted to table_dtype and the MLP copied (and rounded to bf16 for
 * MR_BF16) on the device. */
mr_status mr_field_create(const mr_field_desc* desc, const float* host_table,
                          const float* host_mlp, void* stream, mr_field** out);
mr_status mr_field_destroy(mr_field* f);

/* The MLP weight fragments that mr_field_create stages for the matrix cores
 * (host only: no device is touched).  desc/host_mlp as for mr_field_create
 * (a radiance field).  bf16 != 0: the BF16 engine's fragments (one BF16
 * piece per weight, round to nearest even); bf16 == 0: the FP32 engine's,
 * each weight as three BF16 pieces w0 + w1 + w2 equal to it exactly, stored
 * piece after piece per layer, followed by the FP32 output layer and the
 * FP32 SH columns of colour layer 1.  *words receives the size in 32-bit
 * words; out == NULL asks for the size only.  Otherwise out (host memory of
 * capacity_words words) receives the fragments, or MR_ERR_INVALID_ARG when
 * it is too small.  MR_ERR_UNSUPPORTED for a layout mr_field_create
 * refuses. */
mr_status mr_mlp_fragments(const mr_field_desc* desc, const float* host_mlp, int32_t bf16, uint32_t* out,
                           int64_t capacity_words, int64_t* words);

/* Evaluate the field at n points (device arrays).
 * x, dirs: (n, 3) in world coordinates (mapped into the field's frame when it
 * has a pose); sigma: (n); rgb: (n, 3) or NULL; feat: (n, n_levels*feats)
 * or NULL (interpolated hash features, FP32); raw: (n, density_out) or NULL. */
mr_status mr_field_query(const mr_field* f, int64_t n, const float* x, const float* dirs,
                         float* sigma, float* rgb, float* feat, float* raw, void* stream);

/* Placement of the field in the world, for a moving NeRF object: the field
 * is looked up at R^T (p - c) for a world point p and at R^T d for a world
 * direction d, with host_pose = [R | c] row-major 3x4 (field frame -> world)
 * and R a rotation (R^T R = I within 1e-5, det R = +1; else
 * MR_ERR_INVALID_ARG and the pose is unchanged).  NULL removes the pose.  It
 * applies to renders and queries launched afterwards (a captured graph keeps
 * the pose it was captured with).  The occupancy grid stays in the field's
 * frame; a proposal field is evaluated in the frame of the field it samples
 * for; the proposal training entry points take rays in the field's frame. */
mr_status mr_field_set_pose(mr_field* f, const float* host_pose);

/* Occupancy bit grid for empty-space skipping (attached to the field).
 * Cell (i, j, k) of a res^3 grid over the field box (x fastest) is occupied
 * when sigma >= thresh at any of the centres of its 2x2x2 sub-cells.
 * bits_out: optional device uint8 (res^3) export of the grid.
 * res in 1..512. */
mr_status mr_field_build_occupancy(mr_field* f, int32_t res, float thresh, uint8_t* bits_out,
                                   void* stream);

/* Device pointers of the field's parameters (for training and inspection).
 * table: [L][T][F] in table_dtype; mlp: FP32 flat weights. */
mr_status mr_field_params(mr_field* f, void** table, float** mlp, int64_t* n_table,
                          int64_t* n_mlp);

/* ------------------------------------------------------------------------ */
/* Triangle meshes with per-triangle materials, and their BVH (the surfaces */
/* of Sec. 3.1 "Surface Rendering Equation"; ray casting t(p, w), Eq. 3).   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t kind;      /* MR_MIRROR | MR_GLASS | MR_DIFFUSE */
  float ior;         /* glass index of refraction (> 1) */
  float albedo[3];   /* diffuse reflectance in [0, 1] */
  float emission[3]; /* emitted radiance L_e (linear HDR, >= 0; Eq. 12): every hit adds
                        T L_e with the throughput attenuated by the segment, also when
                        the ray stops there at its bounce limit */
} mr_material;

typedef struct mr_mesh mr_mesh;

/* Build a binary BVH with the surface-area heuristic (binned, on the host)
 * and upload it.  host_vertices (nv, 3); host_indices (nf, 3), each in
 * [0, nv); host_mat_ids (nf) in [0, n_materials).  Triangle ids reported by
 * mr_render are the row numbers of host_indices.  Degenerate (zero-area)
 * triangles are kept and never hit.  Surfaces are two-sided; a triangle's
 * geometric normal is (v1 - v0) x (v2 - v0), and for glass it must point
 * out of the solid. */
mr_status mr_mesh_build_bvh(const float* host_vertices, int32_t nv, const int32_t* host_indices,
                            int32_t nf, const int32_t* host_mat_ids,
                            const mr_material* host_materials, int32_t n_materials,
                            void* stream, mr_mesh** out);

/* Refit the BVH to new vertex positions (device (nv, 3), same topology),
 * bottom-up on the device; no host round trip. */
mr_status mr_mesh_refit(mr_mesh* m, const float* vertices, void* stream);
mr_status mr_mesh_destroy(mr_mesh* m);

/* Statistics of the tree (host values): node count, depth, leaf count. */
mr_status mr_mesh_info(const mr_mesh* m, int32_t* n_nodes, int32_t* depth, int32_t* n_leaves);

/* Closest hit for n rays (device arrays): t in (0, t_max], lexicographic
 * minimum of (t, triangle id).  t_hit (n) = +inf on a miss, tri (n) = -1. */
mr_status mr_mesh_closest_hit(const mr_mesh* m, int64_t n, const float* origins,
                              const float* dirs, float t_max, float* t_hit, int32_t* tri,
                              void* stream);

/* ------------------------------------------------------------------------ */
/* Rendering (Algorithm 1).                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  float pos[3];
  float intensity[3];
} mr_light;

typedef struct {
  float t_near, t_far;       /* camera segment [t_near, t_far]; later segments
                                start at their spawn point with the same length */
  int32_t n_samples;         /* uniform intervals per segment length */
  int32_t sampler;           /* MR_SAMPLER_UNIFORM | MR_SAMPLER_PROPOSAL */
  const mr_field* proposal;  /* proposal field when sampler = PROPOSAL */
  int32_t n_proposal;        /* proposal intervals per segment (32) */
  int32_t n_fine;            /* fine samples drawn from the proposal (32) */
  int32_t use_occupancy;     /* skip empty cells of the field's occupancy grid */
  int32_t rr_after;          /* Russian roulette once this many scatters happened; -1 off */
  float t_min_throughput;    /* terminate when max channel of T drops below (1e-4) */
  uint32_t seed;             /* Philox4x32-10 key */
  int32_t march_blocks_per_cu;  /* launch shape of the persistent march grid: blocks of
                                   4 waves per compute unit (0 = as many as are resident
                                   at once, from the occupancy of the kernel launched) */
  int32_t stage_blocks_per_cu;  /* closest-hit and shade grids: blocks of 128 threads
                                   per compute unit (0 = as many as are resident at once) */
  int32_t stage_tile;           /* rays a block takes per work-queue grab in the
                                   closest-hit and shade stages, a multiple of 128
                                   (0 = default 128) */
  int32_t march_chunk;          /* march ray queue: 0 = one queue for the device; k > 0 =
                                   chunks of k consecutive rays dealt round-robin to the
                                   8 dies (workgroup i runs on die i % 8), each die's
                                   waves taking their own chunks first */
  int32_t march_batch;          /* rays a march wave takes per queue grab, 1..64 (0 = 1) */
  int32_t march_packets;        /* leading bounce segments (uniform sampler) marched as
                                   packets: a wave takes 16 consecutive queue rays and
                                   steps them through the same sample index together, so
                                   rays that are neighbours in the queue and in space
                                   (camera pixels of one image row) share cache lines of
                                   the table; later segments march one ray per wave, 16
                                   samples per tile.  0 = default (1: the caller's rays),
                                   -1 = none, k > 0 = segments 0..k-1 */
  int32_t sample_shadows;       /* 1: shadow mask per field sample (Sec. 3.1 "Shadow
                                   rays"): a ray from each sample to each light, and
                                   every light a mesh hides multiplies the sample's
                                   emitted radiance by shadow_mask (transmittance is
                                   unchanged); both samplers */
  float shadow_mask;            /* mask value of a hidden sample, in [0, 1] (the paper's
                                   1 - r_src, or a constant near 0) */
  int32_t sample_emitters;      /* 1: light sampling toward emitting triangles (Eq. 12's
                                   L_e as area lights): at each diffuse hit one point on one
                                   emitting triangle, the triangle chosen with probability
                                   proportional to its summed emitted radiance and the point
                                   uniform by area; a mesh shadow ray to 0.999 of the way;
                                   the estimate (albedo/pi) L_e cos_p cos_x / d^2 A / p
                                   (emitters two-sided) times the medium's transmittance
                                   along that segment (the fields' density by the midpoint
                                   rule on the march's grid, empty occupancy cells zero;
                                   at most 2^20 grid intervals per field and segment).
                                   A path that reaches an emitter straight after a diffuse
                                   scatter then adds no L_e there.
                                   0: emission only where paths reach it */
  int32_t wait_polls;           /* bound on each wait between the producer and consumer
                                   waves of the packet march, in polls (0 = 2^26, about
                                   seconds).  A wave whose wait runs out stops; the rays of
                                   its packets then miss this segment's medium and
                                   mr_render_status reports it.  Never reached in a correct
                                   run: a bound that keeps every kernel finite */
  int32_t light_depth_samples;  /* with sample_emitters: grid intervals per segment length
                                   for the optical depth along a light sample's shadow
                                   segment (spacing (t_far - t_near) / this), 0..4096;
                                   0 = n_samples, the march's own grid.  Fewer intervals
                                   mean fewer density evaluations per light sample; the
                                   midpoint rule is exact for a constant density */
} mr_render_opts;

/* One launch shape (the launch fields of mr_render_opts). */
typedef struct {
  int32_t march_blocks_per_cu, stage_blocks_per_cu, stage_tile, march_chunk, march_batch, march_packets;
} mr_launch_cfg;

typedef struct {
  float* radiance;           /* (n, 3) linear radiance L */
  float* throughput;         /* (n, 3) throughput T at termination (0 if killed by roulette) */
  int32_t* bounces;          /* (n) number of scattering events */
  int32_t* hit_ids;          /* optional (n, hit_stride): triangle hit by segment s, -1 = none */
  int32_t hit_stride;        /* >= max_bounces + 1 when hit_ids is set */
  int64_t* counters;         /* optional device int64[4]: samples, segments, shadow rays, scatters */
} mr_render_out;

/* Bytes of device workspace mr_render needs for n rays. */
size_t mr_render_workspace_size(int64_t n);

/* Render n rays: origins, dirs (n, 3) device, unit directions.
 * max_bounces >= 0 is the limit on scattering events; per_ray_max_bounces
 * (optional device int32 (n)) overrides it per ray (each <= max_bounces).
 * Each ray marches at most max_bounces + 1 segments.  field NULL = empty
 * medium; mesh NULL = no surfaces.  host_lights: n_lights point lights.
 * workspace: device buffer of mr_render_workspace_size(n) bytes, 256-byte
 * aligned, not shared with a concurrent call.
 * The proposal sampler serves the (8, 4, 1) and (16, 16, 2) layouts; another
 * layout is MR_ERR_UNSUPPORTED.  Every refusal (status other than MR_OK and
 * MR_ERR_DEVICE) comes before the first launch, and then no output or
 * workspace byte is written. */
mr_status mr_render(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                    const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                    const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                    mr_render_out* out, void* workspace, size_t workspace_bytes, void* stream);

/* Status of the last render that used this workspace (mr_render,
 * mr_render_fields or a graph launch): waits for `stream`, writes to
 * *gave_up (optional) the number of packet-march waves whose bounded wait
 * gave up, and returns MR_ERR_DEVICE when it is not 0 (the render's outputs
 * are then incomplete), else MR_OK.  Synchronises with the host. */
mr_status mr_render_status(const void* workspace, int64_t* gave_up, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, hosts that forbid hipMalloc): mr_render without a
 * workspace.  The ray queues and counters live in a fixed device array of
 * the library, MR_NOALLOC_MAX_RAYS * 128 + 4096 bytes (32 MiB + 4 KiB), that
 * every device the library runs on holds until the process ends; the call
 * allocates nothing (the array's address is looked up once per device, on
 * its first call there).  Arguments, outputs, validation and results are
 * those of mr_render, plus:
 *   n <= MR_NOALLOC_MAX_RAYS, else MR_ERR_INVALID_ARG before any launch;
 *   gave_up: optional device int32, set at the end of the render to the
 *   number of packet-march waves whose bounded wait gave up (0 in a correct
 *   run; what mr_render_status reports for mr_render).
 * Every call on one device shares that device's array: calls that overlap
 * on one device (two streams, two threads) race and give wrong results;
 * serialise them.  Stage timing (mr_profile_enable) does not cover it. */
#define MR_NOALLOC_MAX_RAYS 262144
mr_status mr_render_noalloc(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                            const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                            const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                            mr_render_out* out, int32_t* gave_up, void* stream);

/* Several fields in one scene (NeRF objects placed by mr_field_set_pose
 * among the meshes; the paper's dynamic, mesh-aware scenes hold more than one
 * radiance field).  The medium is their sum: density sigma_1 + sigma_2 + ...
 * and colour the density-weighted mean, each field zero outside its box.
 * Under the uniform sampler, fields of one layout (levels, SH components,
 * colour layers, table and MLP types) are marched together over the summed
 * medium: the grid is cut at every box face a segment crosses and each piece
 * sums the fields whose world boxes (aabb under the pose) hold it; their
 * boxes may overlap.  With the proposal sampler, or fields of different
 * layouts, the world boxes must be pairwise disjoint (touching allowed): every
 * field is marched in a pass of its own (with its own proposal) and the
 * passes are composited in the order the ray enters the boxes, which is that
 * sum.  Overlapping boxes there are MR_ERR_UNSUPPORTED, naming the first
 * overlapping pair or the differing layouts.
 * fields: host array of n_fields (1..8) field handles.  proposals: host
 * array of n_fields proposal fields, field k sampled by proposals[k], when
 * opts->sampler is MR_SAMPLER_PROPOSAL (opts->proposal is then not used; a
 * missing list is MR_ERR_INVALID_ARG); NULL for the uniform sampler.  With
 * use_occupancy every field needs its own grid, and a piece is skipped for a
 * field whose grid marks its cell empty.  Other arguments as mr_render;
 * workspace of mr_render_fields_workspace_size(n, n_fields) bytes, which for
 * one field is mr_render_workspace_size(n) (the call is then mr_render). */
size_t mr_render_fields_workspace_size(int64_t n, int32_t n_fields);
mr_status mr_render_fields(const mr_field* const* fields, const mr_field* const* proposals, int32_t n_fields,
                           const mr_mesh* mesh, int64_t n, const float* origins, const float* dirs,
                           int32_t max_bounces, const int32_t* per_ray_max_bounces, const mr_light* host_lights,
                           int32_t n_lights, const mr_render_opts* opts, mr_render_out* out, void* workspace,
                           size_t workspace_bytes, void* stream);

/* HIP-graph capture of one mr_render call: the same arguments (the device
 * buffers are baked into the graph and must stay allocated) are captured once
 * on a private stream into an executable graph; mr_graph_launch replays it on
 * any stream, re-reading the current contents of the input buffers.  Fails
 * with MR_ERR_STATE while kernel timing (mr_profile_enable) is on. */
typedef struct mr_graph mr_graph;
mr_status mr_render_graph_create(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                                 const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                                 const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                                 mr_render_out* out, void* workspace, size_t workspace_bytes, mr_graph** graph);
mr_status mr_graph_launch(mr_graph* graph, void* stream);
mr_status mr_graph_destroy(mr_graph* graph);

/* Launch-shape autotuner: renders the given workload once per candidate
 * launch shape (host array), reps times each after one warm-up, timing with
 * HIP events on stream, and writes the index of the fastest candidate and its
 * mean milliseconds.  The call synchronises with the host.  Output buffers
 * receive the result of the last render; results depend on the launch shape
 * only through march_packets, by FP32 rounding (see mr_autotune_search). */
mr_status mr_autotune_render(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                             const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                             const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                             mr_render_out* out, void* workspace, size_t workspace_bytes,
                             const mr_launch_cfg* host_cands, int32_t n_cands, int32_t reps,
                             int32_t* best_index, float* best_ms, void* stream);

/* The autotuner's own candidate launch shapes for a queue of n rays on the
 * current device (the batched multi-camera wavefront picks its tile and queue
 * sizes from these): per axis, in mr_launch_cfg order (march blocks per CU,
 * stage blocks per CU, stage tile, march chunk, march batch, packet
 * segments), counts[axis] values in values[axis * 6 ...].  counts: host
 * int32[6]; values: host int32[36].  The stage tiles are 128 and those that
 * give each block of an 8-per-CU grid about 16 and 4 grabs of the queue. */
mr_status mr_autotune_candidates(int64_t n, int32_t* counts, int32_t* values);

/* Launch-shape search: coordinate descent over mr_autotune_candidates'
 * values, starting from the launch fields of opts.  Each axis in turn tries
 * each of its values with the other axes held (one warm-up render, then the
 * mean of reps renders timed with HIP events on stream) and keeps the
 * fastest; up to `passes` sweeps over the axes, stopping early when a sweep
 * changes nothing.  Writes the chosen shape, its mean ms, the starting
 * shape's mean ms (start_ms, optional) and the number of shapes timed
 * (n_timed, optional).  The outputs hold the render of the chosen shape.
 * Hit ids and bounces do not depend on the launch shape, nor does radiance
 * except through march_packets: packets composite with a running product per
 * ray and the per-ray march with a prefix product, which round differently
 * (a few ulp).  Synchronises with the host. */
mr_status mr_autotune_search(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                             const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                             const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                             mr_render_out* out, void* workspace, size_t workspace_bytes, int32_t reps,
                             int32_t passes, mr_launch_cfg* best, float* best_ms, float* start_ms,
                             int32_t* n_timed, void* stream);

/* Pinhole camera rays (device output), camera-major, then row-major with the
 * top row first.  host_cams: n_cams records of 12 floats: position (3),
 * look-at (3), up (3), vertical fov in degrees, width, height.  forward =
 * normalize(look_at - pos), right = normalize(up x forward), up' = forward x
 * right; pixel (i, j) looks along forward + u right + v up' with
 * u = (2(i+.5)/W - 1) tan(fov/2) W/H, v = (1 - 2(j+.5)/H) tan(fov/2).
 * capacity >= total pixel count.  Optional per-ray camera index (int32). */
mr_status mr_rays_from_cameras(const float* host_cams, int32_t n_cams, float* origins,
                               float* dirs, int32_t* cam_index, int64_t capacity, void* stream);

/* Per-ray bounce limits from per-camera ones: out[i] = host_cam_limits[cam_index[i]]
 * for n rays (device arrays); cam_index values must be in [0, n_cams). */
mr_status mr_camera_bounce_limits(const int32_t* cam_index, int64_t n, const int32_t* host_cam_limits,
                                  int32_t n_cams, int32_t* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Learned proposal sampler (not in the paper, which marches every segment   */
/* densely; follows the proposal network and loss of Mip-NeRF 360, Barron et */
/* al. 2022).  A proposal field is a radiance-field handle created with      */
/* color_hidden_layers = 0, 5 levels x 2 features, MLP 10 -> 16 -> 1; it     */
/* keeps an FP32 master copy of its table for training.  mr_render with      */
/* sampler = MR_SAMPLER_PROPOSAL takes n_proposal uniform intervals of each  */
/* segment's marching range [lo, hi], weights w_j = T_j alpha_j from the     */
/* proposal density, dilates them to max(w_{j-1}, w_j, w_{j+1}), mixes them */
/* half and half with a uniform density (adding their mean and 1e-3/n), and */
/* places the n_fine fine intervals between the inverse-CDF points          */
/* u = k/n_fine of that piecewise-constant density.                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  float lr, beta1, beta2, eps;
} mr_adam;

/* Training targets from the plain marcher: for each ray (device (n, 3)
 * arrays) march the camera segment [t_near, t_far] clipped to the field box
 * on the uniform n_samples grid without surfaces, and split its weights
 * w_i = T_i alpha_i over n_bins (1..64) equal bins of the clipped range by
 * interval overlap.  lohi (n, 2) receives the range ((0, 0) on a miss),
 * targets (n, n_bins) the histograms. */
mr_status mr_proposal_targets(const mr_field* fine, int64_t n, const float* origins, const float* dirs,
                              float t_near, float t_far, int32_t n_samples, int32_t n_bins, float* lohi,
                              float* targets, void* stream);

/* Proposal loss and its gradient, averaged over n segments: for each segment
 * the proposal weights on n_bins uniform intervals of [lo, hi] against the
 * target histogram, loss sum_j max(0, h_j - w_j)^2 / (h_j + 1e-7).
 * loss: device float; g_table: device FP32 [L][T][F]; g_mlp: device FP32
 * (176).  Both are overwritten.  Uses the FP32 master table. */
mr_status mr_proposal_grad(const mr_field* proposal, int64_t n, const float* origins, const float* dirs,
                           const float* lohi, const float* targets, int32_t n_bins, float* loss,
                           float* g_table, float* g_mlp, void* stream);

/* One Adam step on the FP32 master parameters with the gradient above; the
 * render copy of the table (FP16 or FP32) is refreshed.  Step t (counted
 * per field from 1) sets m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2 and
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), with lr > 0,
 * 0 <= b1, b2 < 1 and eps > 0 (else MR_ERR_INVALID_ARG).  The optimiser
 * state is allocated (hipMalloc) on the first call.  loss: device float. */
mr_status mr_proposal_train_step(mr_field* proposal, int64_t n, const float* origins, const float* dirs,
                                 const float* lohi, const float* targets, int32_t n_bins, const mr_adam* adam,
                                 float* loss, void* stream);

/* ------------------------------------------------------------------------ */
/* Kernel timing for measurement.  While enabled, mr_render records a HIP   */
/* event pair on its stream around each kernel it launches.  mr_profile_read */
/* waits for those events and returns, per stage (0 closest hit, 1 march of */
/* the later segments, 2 shade, 3 march of the camera segment), the summed  */
/* milliseconds and the number of launches,                                 */
/* then clears them.  Process-wide; not for use under graph capture.        */
/* ------------------------------------------------------------------------ */
mr_status mr_profile_enable(int32_t on);
mr_status mr_profile_read(double* ms /*[4]*/, int64_t* launches /*[4]*/);

/* Random-gather ceiling of the memory level that holds a field's hash table
 * (a measurement helper, not part of the method).  Loads about n_loads (>= 8)
 * table entries of f (8 B FP32 / 4 B FP16) at pseudo-random positions in a
 * power-of-two prefix of its [L][T] entries, eight independent loads per lane
 * and round, from a grid of 8 blocks of 256 lanes per compute unit; returns
 * the kernel time in *ms_out (HIP events on `stream`) and the loads actually
 * issued in *loads_out.  sink: one device uint32 the kernel may write.
 * Synchronous (waits for the kernel); not for graph capture.  Fails with
 * MR_ERR_UNSUPPORTED unless the field has 2 features per level. */
mr_status mr_probe_gather(const mr_field* f, int64_t n_loads, uint32_t seed, uint32_t* sink, float* ms_out,
                          int64_t* loads_out, void* stream);

/* The same probe confined to 2^log2_region table entries (8 <= log2_region;
 * the region must lie in the power-of-two prefix of the table).  per_die = 0:
 * every block reads entries [0, 2^log2_region); per_die != 0: block b reads
 * region (b mod 8) of that size, so with workgroups dealt to the eight dies
 * in turn each die reads a region of its own (8 regions must fit).  Gives the
 * gather rate as a function of the working set of each die's L2.  Same
 * outputs and errors as mr_probe_gather, plus MR_ERR_INVALID_ARG for a region
 * that does not fit. */
mr_status mr_probe_gather_region(const mr_field* f, int32_t log2_region, int32_t per_die, int64_t n_loads,
                                 uint32_t seed, uint32_t* sink, float* ms_out, int64_t* loads_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif
