/* fr.h - C ABI of the MI355X differentiable face renderer.
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the render that
 * Dib et al., "Practical Face Reconstruction via Differentiable Ray Tracing"
 * (Eurographics 2021) run in every optimisation step: scene attributes in
 * (geometry, diffuse/specular/roughness reflectance, pose, camera, area
 * lights), image, photometric loss and gradients out (Sec. 4, Eq. energy).
 *
 * Conventions shared by every entry point:
 *  - d_* arguments are DEVICE pointers on the context's device, h_* are host
 *    pointers.  All device buffers are caller-owned, contiguous, FP32 unless
 *    stated, and must stay alive until the work enqueued on `stream` is done.
 *  - Every call only enqueues work on `stream` (a hipStream_t; 0 = the null
 *    stream) and returns without synchronising, except where stated.
 *  - Gradient outputs are ACCUMULATED (+=): callers zero them first.
 *  - Vectors are packed xyz / rgb triples: a "[N*3]" buffer holds N triples.
 *  - Return value: FR_OK or an FR_ERR_* code.  No exception crosses the ABI.
 *    Argument and shape checks are synchronous; device faults surface at the
 *    next synchronising call.  fr_last_error() gives the text of the last
 *    failure on a context.
 */
#ifndef FR_H_
#define FR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* fr_stream; /* == hipStream_t */

enum {
  FR_OK = 0,
  FR_ERR_INVALID_ARG = 1, /* null pointer, bad enum, non-positive size */
  FR_ERR_SHAPE = 2,       /* sizes inconsistent with the mesh or each other */
  FR_ERR_OOM = 3,         /* device allocation failed */
  FR_ERR_BUDGET = 4,      /* serving: request does not fit the HBM budget */
  FR_ERR_DEVICE = 5,      /* a HIP runtime call failed */
  FR_ERR_NONFINITE = 6,   /* serving: a request produced NaN/Inf */
  FR_ERR_LIMIT = 7,       /* BVH deeper than the traversal stack, spp too large, ... */
  FR_ERR_NOT_FOUND = 8    /* serving: unknown request id */
};

/* Mesh update modes of fr_mesh_update. */
enum { FR_REFIT = 0, FR_REBUILD = 1, FR_REBUILD_SAH = 2 };

/* Light shapes.  FR_LIGHT_DIRECTIONAL is a light at infinity (each pixel of
 * the environment map of Sec. 6, "Environment Map vs. Light Stage"): it
 * shines along l = p0 / |p0| (p0 need not be unit; e1, e2 are ignored and
 * get no gradient), `light_rad` is the irradiance it delivers to a surface
 * facing it (radiance times the solid angle the light stands for), a
 * sample receives V rad f_r (n_s . l), and its shadow ray runs over
 * t in (1e-4, 1e4) (the scene must lie well within 1e4).  No random numbers
 * are drawn for it. */
enum { FR_LIGHT_PARALLELOGRAM = 0, FR_LIGHT_TRIANGLE = 1, FR_LIGHT_DIRECTIONAL = 2 };

/* BRDF readings (Appendix A, Eq. brdf_d and Eq. brdf_f).
 * FR_BRDF_PRINTED:   D = (2/r + 2)/(2 pi) (n.h)^(2/r - 2), F = s + (1 - s)(1 - o.h)
 * FR_BRDF_NORMALIZED: D = 1/(pi r) (n.h)^(2/r - 2),      F = s + (1 - s)(1 - o.h)^5 */
enum { FR_BRDF_PRINTED = 0, FR_BRDF_NORMALIZED = 1 };

typedef struct fr_ctx fr_ctx;
typedef struct fr_mesh fr_mesh;

const char* fr_status_string(int status);
const char* fr_last_error(const fr_ctx* ctx);

/* One context per device.  Selects `hip_device` for the calling thread. */
int fr_ctx_create(int hip_device, fr_ctx** out);
int fr_ctx_destroy(fr_ctx* ctx);

/* Triangle mesh of fixed topology (Sec. 3.1: the morphable model keeps its
 * triangulation while the vertices move).
 *  h_tris [n_tris*3] int32 vertex ids, copied.  Builds on the host the
 *  vertex->face adjacency (for normals) and the unique edge list with the
 *  faces beside each edge (for edge sampling); allocates the BVH storage
 *  (one 64-byte node per internal node, one 48-byte record per triangle). */
int fr_mesh_create(fr_ctx* ctx, int32_t n_verts, int32_t n_tris, const int32_t* h_tris, fr_mesh** out);
int fr_mesh_destroy(fr_mesh* mesh);

/* Per-step geometry pass over world-space positions d_verts [N*3]:
 * area-weighted vertex normals (the normal at each vertex, Sec. 3.2), then
 * the BVH.  FR_REBUILD builds it on the GPU (Morton codes, radix sort, binary
 * radix tree, bottom-up boxes); FR_REBUILD_SAH builds it on the host with a
 * binned surface-area heuristic (copies the vertices and triangles to the
 * host; a slower build, a tree that traversal visits less); both then
 * collapse it to the 4-wide traversal tree and SYNCHRONISE to check its
 * depth.  FR_REFIT keeps the last built topology and recomputes boxes only
 * (no synchronisation).  The first update of a mesh must be a rebuild.
 * d_verts must stay unchanged until the renders that use this update have
 * run. */
int fr_mesh_update(fr_mesh* mesh, const float* d_verts, int mode, fr_stream stream);

/* Device pointer to the mesh's current vertex normals [N*3] (valid after an
 * update; owned by the mesh). */
const float* fr_mesh_normals(const fr_mesh* mesh);
/* Unique undirected edges of the mesh (host copy of the table used by the
 * boundary term): h_edges [E*2] vertex ids (lower id first, sorted), h_faces
 * [E*2] adjacent faces (-1 for a border edge).  Pass NULL to query E. */
int32_t fr_mesh_edges(const fr_mesh* mesh, int32_t* h_edges, int32_t* h_faces);
/* Depth of the current BVH (longest root-to-leaf path, in edges). */
int32_t fr_mesh_bvh_depth(const fr_mesh* mesh);

/* Scene of one render (device pointers unless noted).  The lights are the
 * area lights of the virtual light stage (Sec. 3.3), given as polygons:
 * point p0 + a e1 + b e2 with (a,b) in the unit square (parallelogram) or the
 * unit triangle; e1 x e2 points along the emitting side. */
typedef struct {
  int32_t width, height;   /* image size in pixels */
  int32_t spp;             /* samples per pixel: a power of two, 1..1024 */
  int32_t n_lights;
  const float* verts;      /* [N*3] world positions; same buffer as fr_mesh_update */
  const float* diffuse;    /* [N*3] per-vertex diffuse albedo c_i (Sec. 3.2) */
  const float* specular;   /* [N*3] per-vertex specular albedo s_i */
  const float* roughness;  /* [N] per-vertex roughness r_i (clamped to [1e-3,1] in shading) */
  const float* light_p0;   /* [L*3] */
  const float* light_e1;   /* [L*3] */
  const float* light_e2;   /* [L*3] */
  const float* light_rad;  /* [L*3] RGB radiance */
  const int32_t* light_shape; /* [L] FR_LIGHT_* (device) */
  const float* cam;        /* [12] camera-to-world rotation R (row-major 3x3), then centre T */
  float fov_y;             /* vertical field of view, radians (host value) */
  uint32_t step;           /* optimisation step: the 4th Philox counter word */
  uint64_t seed;           /* Philox key */
  /* Reflectance maps (Sec. 3.2: diffuse, specular and roughness as M x M
   * images in texture space).  tex_size M > 0 selects them in place of the
   * per-vertex diffuse/specular/roughness (which may then be NULL); M = 0
   * leaves the per-vertex arrays in use and the pointers below unread.
   * A shading point takes (u, v) = sum_k b_k uv_k over the hit triangle's
   * corners and reads each map bilinearly: texel (i, j) is centred at
   * ((i + 1/2)/M, (j + 1/2)/M), addresses clamp to the border texel.
   * All device pointers, read only, M <= 16384. */
  int32_t tex_size;
  int32_t tex_pad_;
  const float* tex_uv;        /* [F*3*2] (u, v) of each triangle corner, in triangle order */
  const float* tex_diffuse;   /* [M*M*3] texel (i, j) at offset 3 (j M + i) */
  const float* tex_specular;  /* [M*M*3] */
  const float* tex_roughness; /* [M*M] */
  /* Spherical-harmonics lighting (Sec. 6, "Spherical Harmonics (SH) vs.
   * Light Stage"): a distant light given by the real SH coefficients L_lm
   * of its radiance, bands l < sh_bands (0 = none, at most 11), z the polar
   * axis, sh [B*B*3] at index l(l+1)+m with RGB inner (device).  It adds,
   * on top of the lights and without visibility, (c / pi) E(n_s) to every
   * shaded sample, E(n) = sum_l A_l sum_m L_lm Y_lm(n) the irradiance of the
   * clamped cosine (A_0 = pi, A_1 = 2 pi / 3, A_2 = pi / 4, ...), on the
   * diffuse term only. */
  const float* sh;
  int32_t sh_bands;
  int32_t sh_pad_;
} fr_scene;

typedef struct {
  int32_t brdf_variant;    /* FR_BRDF_* */
  int32_t components;      /* bit 0 diffuse, bit 1 specular (3 = full BRDF) */
  int32_t edge_samples;    /* boundary-term samples in the backward; 0 = off, -1 = W*H */
  int32_t light_chunk;     /* lights per work item, 0..32 (0 = library default per pass; the
                            * backward takes at least ceil(n_lights / 4)) */
  /* Debug dump of the decisions (device, nullable):
   *   dbg_hit [W*H*spp] int32 closest-hit triangle id per sample (-1 = miss);
   *   dbg_pflag [W*H*spp] uint8 nonzero when that decision is near ambiguous;
   *   dbg_vis [W*H*spp*L] uint8 light code 0 occluded, 1 visible, 2 culled,
   *     3 no shading point, ORed with 0x80 when near ambiguous.
   * Sample order is pixel-major: index (y*W + x)*spp + s.
   * In fr_render_backward the dump covers the boundary term instead (dbg_vis
   * must be NULL): dbg_hit [n_edge_samples*4] receives per edge sample the
   * edge id, the pixel id (-1 outside the image) and the hit triangle of the
   * minus and plus side rays; dbg_pflag [n_edge_samples] its ambiguity flag,
   * OR-accumulated (the caller zeroes it). */
  int32_t* dbg_hit;
  uint8_t* dbg_pflag;
  uint8_t* dbg_vis;
  /* Traversal statistics of the forward dump (device, nullable, accumulated):
   * [11] uint64: for camera rays, the child boxes a single-ray traversal of
   * each ray tests (the children of every 4-wide node its ray enters), its
   * triangle tests, and the rays traced; the same three for shadow rays;
   * then the node visits and leaf visits executed by the wave packets for
   * camera rays, then for shadow rays; then the camera samples that reach a
   * shading point (a hit facing the camera). */
  uint64_t* dbg_stats;
  /* Timing (nullable): two hipEvent_t recorded on the stream immediately
   * before the primary pass (the camera rays of every sample; the main
   * kernel, when the backward reuses the forward's hits) and after the
   * main render kernel of the call (the forward render kernel, or the
   * interior adjoint kernel of fr_render_backward). */
  void* ev_kernel_begin;
  void* ev_kernel_end;
  /* fr_render_backward only: nonzero takes the camera-ray hits of every
   * sample from the last render call on this mesh instead of tracing them
   * again, when that call matches this one: same width, height, spp, seed,
   * step, fov_y, vertex buffer, camera buffer, and no fr_mesh_update since;
   * and, when that call was a forward with keep_shadows set and the light
   * buffers (light_p0, light_e1, light_e2, light_shape) and n_lights match
   * too, its shadow decisions instead of tracing the shadow rays.  The
   * caller vouches that the contents of those buffers are unchanged since
   * then (the library compares pointers, not contents).  On any mismatch the
   * backward traces what it cannot take.  Forward and backward with the same
   * counters make identical decisions, so the gradients are bit-identical
   * either way. */
  int32_t reuse_forward;
  /* fr_render_forward only: nonzero also keeps the shadow decision of every
   * sample and light (one bit each, in the workspace: 4 bytes per sample and
   * chunk of light_chunk lights) for a backward with reuse_forward. */
  int32_t keep_shadows;
  /* fr_render_forward only: how the shadow rays walk the tree.  0: the wave
   * packet (the 64 lanes of a wave share one traversal order, nodes fetched
   * by scalar loads; the default and the faster); 1: each lane walks alone
   * (its own stack and vector loads).  The same results either way; ignored
   * by debug dumps.  Other values: FR_ERR_INVALID_ARG. */
  int32_t shadow_traversal;
  /* Device scratch of the call (required): caller-owned device memory on the
   * mesh's device, 256-byte aligned, at least the bytes
   * fr_render_workspace_size gives for this scene and options.  No render
   * call allocates device memory.  The workspace also carries a forward's
   * decisions (camera-ray hits, kept shadow masks) to a backward with
   * reuse_forward: pass both calls the same workspace.  Calls that may run at
   * the same time (other streams, other threads) need distinct workspaces;
   * with distinct workspaces, calls on one mesh may overlap (the mesh is only
   * read by render calls; fr_mesh_update must not overlap them). */
  void* workspace;
  size_t workspace_bytes;
} fr_render_opts;

/* Gradients of a backward pass; every pointer is nullable ("not requested")
 * and accumulated into. */
typedef struct {
  float* verts;      /* [N*3] world positions (includes the path through the normals) */
  float* normals;    /* [N*3] dE/dn of the vertex normals (intermediate; nullable) */
  float* diffuse;    /* [N*3] */
  float* specular;   /* [N*3] */
  float* roughness;  /* [N] */
  float* light_geom; /* [L*9] p0, e1, e2 */
  float* light_rad;  /* [L*3] */
  float* cam;        /* [12] R row-major, T */
  /* reflectance maps (scene tex_size M > 0; untouched otherwise); with maps
   * in use the per-vertex diffuse/specular/roughness receive nothing */
  float* tex_diffuse;   /* [M*M*3] */
  float* tex_specular;  /* [M*M*3] */
  float* tex_roughness; /* [M*M] */
  float* sh;            /* [B*B*3] SH coefficients (fr_scene.sh_bands > 0) */
} fr_grads;

/* Bytes of the workspace (fr_render_opts.workspace) that fr_render_forward,
 * fr_render_backward and fr_shadow_edges need for scenes of this size
 * (width, height, spp, n_lights, tex_size, sh_bands) under these options
 * (light_chunk; keep_shadows adds the forward's kept shadow masks) on this
 * mesh.  One workspace of this size serves all three calls.  Sec. 4 Eq.
 * energy: the render and its gradient, whose per-call state (camera-ray hits,
 * light table, partial images, fixed-point gradient sums) lives here.
 * FR_ERR_INVALID_ARG on a null pointer or a non-positive size. */
int fr_render_workspace_size(const fr_mesh* mesh, const fr_scene* scene, const fr_render_opts* opts, size_t* bytes);

/* Forward render (Sec. 4 Eq. energy: p^S = F(chi), the Monte-Carlo estimate
 * of the rendering equation with direct light only, shadows by shadow rays,
 * Sec. 3.3 "Shadows approximation"; Cook-Torrance BRDF of Appendix A).
 * Per pixel (x,y) and sample s, Philox4x32-10 with key `seed` and counter
 * (y*W + x, s, purpose, step) gives the film jitter (purpose 0) and one point
 * on each light j (purpose 1 + j); one shadow ray per light and sample.
 * d_image [H*W*3] receives the pixel means (row-major, y = 0 at the top). */
int fr_render_forward(fr_mesh* mesh, const fr_scene* scene, const fr_render_opts* opts, float* d_image,
                      fr_stream stream);

/* Photometric loss (Sec. 4 Eq. energy and "Variance Reduction"): optional
 * 3x3 Gaussian smoothing (sigma 1, clamp-to-edge) of d_image, then
 * E = sum |p~ - p^R| over pixels and channels (FP64 accumulation in a fixed
 * order).  d_loss [1] float receives E (overwritten); d_dEdp [H*W*3]
 * (nullable) receives dE/dp = K^T * sign(p~ - p^R) (overwritten).  d_work:
 * caller-owned device scratch, 256-byte aligned, of at least
 * fr_loss_workspace_size(width, height, smooth) bytes (FR_ERR_SHAPE if
 * smaller); calls that may overlap need distinct scratch. */
size_t fr_loss_workspace_size(int32_t width, int32_t height, int32_t smooth);
int fr_loss(const float* d_image, const float* d_target, int32_t width, int32_t height, int32_t smooth,
            float* d_loss, float* d_dEdp, void* d_work, size_t work_bytes, fr_stream stream);

/* fr_loss for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation, arguments and results, with the scratch in a static device
 * array of the library instead of a caller workspace.  The array holds the
 * scratch of images of at most 2^20 pixels (1024 x 1024; 12.6 MB per device,
 * resolved at fr_ctx_create or at the first call on a device and held until
 * the process ends); larger images return FR_ERR_LIMIT before any launch.
 * Every call on a device shares that device's array (each call writes all the
 * scratch it reads, so nothing carries over between calls): calls that
 * overlap in time on one device race; serialise them on one stream.
 * FR_ERR_DEVICE if the runtime cannot give the array's address. */
int fr_loss_noalloc(const float* d_image, const float* d_target, int32_t width, int32_t height, int32_t smooth,
                    float* d_loss, float* d_dEdp, fr_stream stream);

/* Stage II regularisers of the personalised reflectance maps (Sec. 4
 * "Stage II", Eq. loss3; the paper's weights are w_sym = w_chroma = 0.3,
 * w_smooth = 0.0002, w_box = 1):
 *   w_sym (E_s(C) + E_s(S)) + w_chroma (E_c(C, C0) + E_c(S, S0))
 *   + w_smooth (E_m(C) + E_m(S) + E_m(R)) + w_box (E_b(S) + E_b(R))
 * over M x M maps (C, S, C0, S0 [M*M*3], R [M*M], texel (i, j) at j M + i,
 * device): E_s the L1 difference to the horizontally flipped map (i to
 * M - 1 - i), E_c the L1 difference of chromaticities x / (x_r + x_g + x_b +
 * 1e-6) to the Stage I maps C0, S0, E_m the squared differences of each
 * texel to its in-map 4-neighbours, E_b the squared excess outside [0, 1].
 * d_loss [1] float is overwritten (FP64 sums in a fixed order); the
 * gradients (nullable) are accumulated (+=).  d_work: caller-owned device
 * scratch, 256-byte aligned, of at least fr_map_regularizers_workspace_size(M)
 * bytes (FR_ERR_SHAPE if smaller). */
typedef struct { float w_sym, w_chroma, w_smooth, w_box; } fr_map_reg_weights;

/* Stage I priors (Sec. 4 "Stage I", Eq. loss1; Sec. 5 weights w_i = w_c =
 * w_s = 0.0025, w_1 = 0.01), over n device floats d_x:
 *   FR_PRIOR_STATISTICAL  weight sum (x_k / sigma_k)^2 (d_sigma [n]);
 *   FR_PRIOR_BOX          weight sum (min(x, 0)^2 + max(x - 1, 0)^2);
 *   FR_PRIOR_LIGHT_CHROMA weight sum_j ||I_j - mean_c I_j||^2 over the n / 3
 *                         RGB intensities I_j (d_sigma unused).
 * d_loss [1] float is overwritten (FP64 sums in a fixed order, one
 * workgroup: meant for parameter vectors, not images); d_g (nullable)
 * += dE/dx.  No scratch memory. */
enum { FR_PRIOR_STATISTICAL = 0, FR_PRIOR_BOX = 1, FR_PRIOR_LIGHT_CHROMA = 2 };

/* Landmark loss (Sec. 4 Eq. landmark): sum_l || Pi(v_l) - z_l ||^2 over n
 * landmarks, v_l = d_verts[d_idx[l]] (world positions, distinct indices),
 * Pi the render's pinhole (Sec. 3.1; cam [12] as in fr_scene, fov_y and
 * the W x H image: film points in pixels, y down), z_l = d_z [n*2].
 * d_loss [1] float overwritten; d_gverts [N*3] and d_gcam [12] (nullable)
 * accumulate (+=). */
int fr_landmark_loss(const float* d_verts, const int32_t* d_idx, int32_t n, const float* d_cam, float fov_y, int32_t W,
                     int32_t H, const float* d_z, float* d_loss, float* d_gverts, float* d_gcam, fr_stream stream);
int fr_prior(const float* d_x, const float* d_sigma, int32_t n, int32_t kind, float weight, float* d_loss, float* d_g,
             fr_stream stream);
size_t fr_map_regularizers_workspace_size(int32_t M);
int fr_map_regularizers(const float* d_c, const float* d_s, const float* d_r, const float* d_c0, const float* d_s0,
                        int32_t M, const fr_map_reg_weights* weights, float* d_loss, float* d_gc, float* d_gs,
                        float* d_gr, void* d_work, size_t work_bytes, fr_stream stream);

/* Backward pass: the adjoint of fr_render_forward for a given dE/dp
 * d_dEdp [H*W*3], recomputing every intersection and shadow decision from the
 * same counters (or taking the forward's, opts->reuse_forward) and holding
 * them fixed (interior term),
 * then the vertex-normal adjoint into grads->verts, then, if
 * opts->edge_samples != 0, the primary-visibility boundary term of edge
 * sampling (Sec. 4 "Edge Sampling") into grads->verts and grads->cam.
 * With reflectance maps each shading point spreads its reflectance gradient
 * over its four texels by the bilinear weights (grads->tex_*), and the maps'
 * own slope in (u, v) carries into the barycentrics and the vertices.
 * Any number of lights: more than 128 are taken in groups of 128, one
 * adjoint and one boundary-term launch per group (the sample-level chain
 * is linear in the summed per-light adjoints, so the groups' chains add).
 * Scratch and the forward's decisions come from opts->workspace.
 * Streams: the boundary term runs on a second stream that the mesh creates
 * at its first backward (default priority; destroyed with the mesh), forked
 * from `stream` after the accumulators are zeroed and joined back before
 * the conversions, by events; the call stays ordered on `stream` (also
 * under stream capture, where the fork and join are captured as graph
 * edges), and backward calls on one mesh from several threads serialise
 * their enqueue.  The gradients are fixed-point integer sums, so they do
 * not depend on how the two streams interleave. */
int fr_render_backward(fr_mesh* mesh, const fr_scene* scene, const fr_render_opts* opts, const float* d_dEdp,
                       fr_grads* grads, fr_stream stream);

/* Shadow-edge (secondary visibility) boundary term of the adjoint (Sec. 4
 * "Edge Sampling", for the visibility of the shadow rays of Sec. 3.3):
 * n_samples line samples, accumulated (+=) into grads->verts, ->light_geom
 * and ->cam (the other fields are ignored; each pointer nullable).  Light j
 * seen from a shading point x contributes kappa^-1 int int h V dw1 dw2 over
 * its parameters (y = p0 + w1 e1 + w2 e2; kappa = 1 parallelogram, 1/2
 * triangle; h the render's per-sample light value).  Samples come in groups
 * of 64: group g draws, from Philox counter (g, 0, 0xC0000000, step), an
 * 8 x 8 pixel tile (word 0: floor(r n_tiles / 2^32); tiles at the right and
 * bottom borders are clipped to the image) and a light (word 1, the same
 * rule over n_lights); sample i of the group draws, from counter (i, 1,
 * 0xC0000000, step), a camera sample among the tile's pixels and samples
 * (word 0) and the line w2 = v (word 1, its top 24 bits).  Each sample traces
 * its camera ray and adds, for each jump w1_k of V along the line (an
 * occluder edge crossing the wedge from x to the line, its faces other than
 * x's triangle on one side as seen from x, the shadow ray to y(w1_k, v)
 * otherwise free), kappa^-1 (1/spp) (dEdp[pixel] . h) J_k dw1_k/dtheta /
 * (n_samples p), J_k = V(w1_k-) - V(w1_k+), p = p(tile) p(camera sample |
 * tile) p(light), each the exact probability of its draw (the count of
 * 32-bit words that select it, over 2^32).  Lights at infinity contribute
 * nothing here (their shadows are hard: a screen-space term, not built); nor
 * does a sample whose light is wholly below x's tangent plane (every corner
 * 1e-4 below) or whose x is behind the light (1e-3 of its area-normal size):
 * h = 0 on its line, so it records no jumps and skips the walk.  Manifold
 * meshes (an edge with more than two faces is not supported).  Call after
 * fr_mesh_update of the same vertices (the walk uses the mesh's tree).
 * d_dEdp [H*W*3] device.  d_rec [n*4] / d_flag [n] (nullable, together):
 * per sample (camera sample, light, jumps that passed the occlusion test,
 * sum of their edges' lower vertex id * N + upper id, mod 2^31) and 1 when a
 * decision was near-ambiguous.  Requires W*H*spp < 2^31 (FR_ERR_LIMIT).
 * Scratch from opts->workspace (a forward's kept decisions there stay). */
int fr_shadow_edges(fr_mesh* mesh, const fr_scene* scene, const fr_render_opts* opts, const float* d_dEdp,
                    int32_t n_samples, fr_grads* grads, int32_t* d_rec, uint8_t* d_flag, fr_stream stream);

/* Morphable blend (Sec. 3.1, Sec. 3.2): d_out[m] = d_mean[m] + sum_k
 * d_coef[k] d_basis[k*M + m], m < M, with the basis stored component-major
 * ([K][M]).  Geometry: mean = a_s, basis = [Sigma_s; Sigma_e], coef =
 * [alpha; delta]; albedo: a_r, Sigma_r, beta. */
int fr_blend(const float* d_mean, const float* d_basis, const float* d_coef, int32_t K, int32_t M, float* d_out,
             fr_stream stream);
/* Adjoint of fr_blend: d_gcoef[k] += sum_m d_basis[k*M + m] d_gout[m]. */
int fr_blend_backward(const float* d_basis, const float* d_gout, int32_t K, int32_t M, float* d_gcoef,
                      fr_stream stream);

/* Rigid pose of the mesh: d_vw = R v + t with R = Rz(rz) Ry(ry) Rx(rx),
 * d_pose [6] = (rx, ry, rz, tx, ty, tz) (the rotation/translation of
 * Sec. 3.1 applied to the object; the camera keeps its own R, T). */
int fr_pose_forward(const float* d_v, int32_t n_verts, const float* d_pose, float* d_vw, fr_stream stream);
/* Adjoint: d_gv [N*3] += R^T d_gw (nullable), d_gpose [6] += dE/dpose. */
int fr_pose_backward(const float* d_v, int32_t n_verts, const float* d_pose, const float* d_gw, float* d_gv,
                     float* d_gpose, fr_stream stream);

/* Virtual light stage (Sec. 3.3 "Virtual Light Stage", Eq. lightIntensity):
 * light j lives on face j of a convex base shape (d_faces [J*9]: its three
 * vertices; the icosahedron of unit circumradius, 20 faces, in the paper),
 * with parameters d_params [J*7] = (d, a, p1, p2, i_r, i_g, i_b): the face
 * scaled about the origin so that its centroid lies at distance d (the
 * homothetic face); a triangle light similar to it with a times its area,
 * centred at barycentric position (p1, p2) within it, parallel to it and
 * emitting towards the origin; radiance I = d^2 / a * i.  Writes the
 * triangle lights of fr_scene: d_p0, d_e1, d_e2, d_rad [J*3] and
 * d_shape [J] = FR_LIGHT_TRIANGLE (each nullable).  a > 0 and d > 0 are the
 * caller's (the paper keeps them there by a soft box constraint). */
int fr_light_stage(const float* d_faces, const float* d_params, int32_t n_lights, float* d_p0, float* d_e1,
                   float* d_e2, float* d_rad, int32_t* d_shape, fr_stream stream);
/* Adjoint: d_gparams [J*7] += the gradient of sum(g_geom . (p0, e1, e2)) +
 * sum(g_rad . rad), with d_g_geom [J*9] (p0, e1, e2: the light_geom layout
 * of fr_grads) and d_g_rad [J*3] (each nullable). */
int fr_light_stage_backward(const float* d_faces, const float* d_params, int32_t n_lights, const float* d_g_geom,
                            const float* d_g_rad, float* d_gparams, fr_stream stream);

/* A per-vertex attribute written into an M x M texture map: the Stage II
 * maps start from the Stage I statistical albedo read in texture space
 * (Sec. 4 "Stage II").  d_tris [F*3] vertex ids and d_uv [F*3*2] per-corner
 * texture coordinates (the layout of fr_scene.tex_uv), d_attr [N*channels]
 * (channels 1..4), d_map [M*M*channels], texel (i, j) at j M + i.  Texel
 * (i, j) with centre c = ((i + 1/2)/M, (j + 1/2)/M) inside the texture
 * triangle of face f receives sum_k b_k attr[tris[f][k]] (b the barycentrics
 * of c); a centre on an edge or vertex belongs to one face only (each edge
 * function positive, or zero on a left or top edge of the counter-clockwise
 * triangle, edges evaluated from their lexicographically lower end); texels
 * that no face holds are left as they are.  FP64 arithmetic.  Device
 * pointers. */
int fr_bake_vertex_map(const int32_t* d_tris, const float* d_uv, int32_t n_tris, const float* d_attr, int32_t channels,
                       int32_t M, float* d_map, fr_stream stream);

/* d_y[i] += a * s * d_x[i], i < n, with s = d_s[0] (a device scalar, e.g. the
 * upstream gradient of a loss) or 1 when d_s is NULL: how an optimisation
 * step adds up the terms of its objective (Sec. 4 Eq. loss1, Eq. loss3) and
 * their gradients on the device.  Device pointers; d_y and d_x must not
 * overlap unless equal. */
int fr_axpy(float* d_y, const float* d_x, float a, const float* d_s, int32_t n, fr_stream stream);

/* Adam (Sec. 5 "Implementation Details": beta1 0.9, beta2 0.999, one learning
 * rate per parameter group), step number t >= 1, per-element learning rate
 * d_lr [n]: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
int fr_adam_step(float* d_param, const float* d_grad, float* d_m, float* d_v, const float* d_lr, int32_t n,
                 int32_t t, float beta1, float beta2, float eps, fr_stream stream);

/* ---------------------------------------------------------------------------
 * Batched reconstructions.  A model holds what every reconstruction of a face
 * shares: the mesh topology and the morphable model of Sec. 3.1 / 3.2 (device
 * pointers, caller-owned, kept alive while the model is used).  A job is one
 * reconstruction: its parameters [alpha, delta | beta | pose(6) | radiance
 * (3L)] are optimised with Adam (Sec. 5) against its target image, with its
 * own image size, samples per pixel and lights.  fr_batch_step advances every
 * job of a batch by one or more optimisation steps (blend, pose, normals +
 * refit, render, loss, backward with edge sampling and, for a job that asks
 * for it, the shadow-edge term, adjoints, Adam), with one launch per stage covering all jobs; with use_graph the launch sequence is
 * captured into a hipGraph once per job set and replayed.
 * ------------------------------------------------------------------------- */
typedef struct fr_model fr_model;
typedef struct fr_batch fr_batch;

typedef struct {
  int32_t width, height, spp, n_lights;
  int32_t edge_samples;    /* boundary-term samples per step: -1 = W*H, 0 = off */
  int32_t smooth;          /* 1: 3x3 Gaussian smoothing before the loss */
  int32_t brdf_variant;    /* FR_BRDF_* */
  int32_t hist_cap;        /* per-step losses kept on the device */
  uint64_t seed;           /* Philox key of this job's renders */
  float fov_y;             /* host value, radians */
  int32_t shadow_edge_samples; /* line samples per step of the shadow-edge boundary term
                                  (Sec. 4 "Edge Sampling" on the shadow rays of Sec. 3.3; the
                                  fr_shadow_edges estimator, vertex gradients only):
                                  0 = off, -1 = W*H */
  /* host or device memory, copied at fr_batch_add (free to reuse afterwards): */
  const float* cam;        /* [12] camera R (row-major), T */
  const float* light_p0;   /* [L*3] */
  const float* light_e1;   /* [L*3] */
  const float* light_e2;   /* [L*3] */
  const int32_t* light_shape; /* [L] */
  const float* target;     /* [H*W*3] target image p^R */
  const float* params;     /* [n_param] initial parameters */
  const float* lr;         /* [n_param] per-parameter learning rates */
} fr_job_desc;

int fr_model_create(fr_ctx* ctx, int32_t n_verts, int32_t n_tris, const int32_t* h_tris, const float* d_mean_geo,
                    const float* d_basis_geo, int32_t K_geo, const float* d_mean_alb, const float* d_basis_alb,
                    int32_t K_alb, const float* d_specular, const float* d_roughness, fr_model** out);
int fr_model_destroy(fr_model* model);
/* Parameters of a job with n_lights lights: K_geo + K_alb + 6 + 3 n_lights. */
int32_t fr_model_n_param(const fr_model* model, int32_t n_lights);
/* Device bytes one job of this description occupies (its mesh, BVH and
 * buffers); the serving loop admits jobs against an HBM budget with it. */
size_t fr_job_bytes(const fr_model* model, const fr_job_desc* desc);

int fr_batch_create(fr_model* model, fr_batch** out);
int fr_batch_destroy(fr_batch* batch);
/* Allocate a job, copy its inputs, build its BVH (synchronises). */
int fr_batch_add(fr_batch* batch, const fr_job_desc* desc, int32_t* job_id, fr_stream stream);
/* Free a job (synchronises the device first). */
int fr_batch_remove(fr_batch* batch, int32_t job_id);
int32_t fr_batch_size(const fr_batch* batch);
/* n_steps optimisation steps of every job (Sec. 4: blend, pose, refit,
 * render, loss, adjoint with its boundary terms, pose and blend adjoints,
 * Adam), one launch per stage for all jobs.  use_graph != 0: the launch
 * sequence is captured into a hipGraph at the first step after the job set
 * changes and replayed.  Part of each step runs on a second stream of the
 * batch (default priority), forked from and joined back to `stream` by
 * events, so the call stays ordered on `stream`.  Asynchronous. */
int fr_batch_step(fr_batch* batch, int32_t n_steps, int32_t use_graph, fr_stream stream);
/* Copy a job's state to host buffers (each nullable): parameters [n_param],
 * gradient of the last step [n_param], per-step losses [hist_cap] (loss of the
 * image rendered at step k in entry k - 1), last rendered image [H*W*3],
 * completed steps.  Synchronises the stream. */
int fr_batch_read(fr_batch* batch, int32_t job_id, float* h_params, float* h_grad, float* h_loss_hist,
                  float* h_image, int32_t* h_t, fr_stream stream);

/* Size of a job and its completed steps. */
int fr_batch_job_info(const fr_batch* batch, int32_t job_id, int32_t* n_param, int32_t* hist_cap,
                      int32_t* steps_done);
/* Latest loss of every job (at most cap, in job-id order) into h_ids / h_losses;
 * returns the count, or -FR_ERR_* on failure.  Synchronises the stream. */
int32_t fr_batch_losses(fr_batch* batch, int32_t cap, int32_t* h_ids, float* h_losses, fr_stream stream);

/* ---------------------------------------------------------------------------
 * Serving.  A server owns a worker thread, a HIP stream and a batch on the
 * model's device, and runs submitted reconstructions with continuous
 * batching: between optimisation steps it admits queued requests in arrival
 * order while a slot is free, the request's device bytes (fr_job_bytes)
 * fit the HBM budget and its rays per step fit the work cap, steps all admitted requests together, fails a request
 * whose loss turns non-finite (FR_ERR_NONFINITE), and retires the ones that
 * reached their step count.  A request is never split or preempted; a request
 * that does not fit the remaining budget blocks those behind it (strict FIFO).
 * All calls are thread-safe and return at once except fr_server_wait.
 * ------------------------------------------------------------------------- */
typedef struct fr_server fr_server;

typedef struct {
  size_t hbm_budget;     /* device bytes the admitted requests may hold together */
  int32_t max_slots;     /* requests stepped together at most */
  int32_t quantum;       /* steps per scheduling round at most (bounds admission delay) */
  int32_t use_graph;     /* 1: replay each round's step from a hipGraph */
  int32_t pad_;
  double work_cap;       /* nominal rays per step (width*height*spp*(1+lights), summed over
                            the admitted requests) admitted together at most; <= 0: no cap.
                            The request at the head of the queue is admitted whenever
                            nothing runs, whatever its work. */
} fr_server_opts;

typedef struct {
  fr_job_desc job;       /* pointers: HOST memory, copied at submit */
  int32_t n_steps;       /* Adam steps to run */
  int32_t pad_;
} fr_request;

enum { FR_REQ_QUEUED = 0, FR_REQ_RUNNING = 1, FR_REQ_DONE = 2, FR_REQ_FAILED = 3, FR_REQ_CANCELLED = 4 };

typedef struct {
  int32_t state;         /* FR_REQ_* */
  int32_t status;        /* FR_OK, or why the request failed */
  int32_t steps_done, n_steps, n_losses;
  float final_loss;      /* loss of the image rendered at the last step run */
  double t_submit, t_admit, t_done;   /* seconds on the server clock */
} fr_result;

typedef struct {
  int64_t submitted, completed, failed, cancelled, rejected;
  int32_t queued, active, peak_active, pad_;
  size_t bytes_in_use, peak_bytes;
  double p50_s, p99_s, mean_s;   /* arrival-to-done latency of completed requests (nearest rank) */
  double recons_per_s;           /* completed / (last completion - first arrival) */
  double busy_s;                 /* time spent in batched steps */
  int64_t steps, ticks;          /* batched steps run, scheduling rounds */
} fr_stats;

int fr_server_create(fr_model* model, const fr_server_opts* opts, fr_server** out);
/* Stops the worker; requests still queued or running are dropped. */
int fr_server_destroy(fr_server* server);
/* FR_ERR_BUDGET if the request alone exceeds the budget. */
int fr_server_submit(fr_server* server, const fr_request* req, uint64_t* id);
/* State of a request; when done (or failed after running) also its final
 * parameters [n_param] and per-step losses [n_steps] (both nullable). */
int fr_server_poll(fr_server* server, uint64_t id, fr_result* out, float* h_params, float* h_losses);
int fr_server_cancel(fr_server* server, uint64_t id);
/* Drop the record of a finished request. */
int fr_server_forget(fr_server* server, uint64_t id);
int fr_server_stats(fr_server* server, fr_stats* out);
/* Block until nothing is queued or running: FR_OK, or FR_ERR_LIMIT after timeout_s. */
int fr_server_wait(fr_server* server, double timeout_s);
/* Seconds since the server was created (the clock of fr_result). */
double fr_server_clock(fr_server* server);

/* ---------------------------------------------------------------------------
 * Measurement probe (not part of the render): `blocks` workgroups of 256
 * lanes each run eight independent FP32 FMA chains of `iters` steps (8 *
 * iters lane-FMAs per lane, no memory traffic but one store per lane into
 * d_out [blocks*256]).  Timed by the caller, it gives the achievable rate of
 * the non-packed FP32 lane-operations that the ALU roofline of the render
 * kernels counts.
 * ------------------------------------------------------------------------- */
int fr_probe_valu(int32_t blocks, int32_t iters, float* d_out, fr_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* FR_H_ */
