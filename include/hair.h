/*
 * hair.h -- C-ABI of the MI355X level-of-detail strand-hair renderer (libhair.so).
 *
 * Method: "Real-time Level-of-detail Strand-based Hair Rendering" (arxiv 2405.10565).
 *   - strands and their elliptical thick-hair (cluster) levels:        Sec. 5.1
 *   - per-frame hair width and level choice (eps_w = 2 px):            Sec. 5.1 step 5, 5.2, 6
 *   - single-fibre scattering f = sum_p A_p M_p N_p (R/TT/TRT, R/TT/D): Sec. 3.1 (eq. bcsdf)
 *   - aggregated thick-hair scattering f_ours:                         Sec. 4 (eq. our_bcsdf)
 *   - radiance L = sum_lights E f cos(theta_i):                        Sec. 3 (rendering eq.)
 * Segments are binned into 16x16-pixel tiles, covered on a 1/16-pixel integer grid, shaded
 * per fragment and composited per pixel front to back in (depth key, segment id) order.
 *
 * Conventions for every entry point:
 *   - return value: HAIR_OK (0) or a negative HAIR_E* code; on error nothing the caller owns
 *     has been written and hair_last_error() describes the failure (thread-local string).
 *   - "host" pointers are read (or written) before the call returns; "device" pointers must
 *     stay valid until the work enqueued on `stream` completes.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every kernel of a call
 *     runs on it; calls that read results back to the host synchronise it.
 *   - memory the library allocates (assets, LoD levels, workspaces) counts against the
 *     context's HBM budget; exceeding it returns HAIR_ENOMEM and allocates nothing.
 *   - a context may be used from several threads; renders on distinct workspaces may run
 *     concurrently.  One workspace serves one call at a time, and a workspace holding a frame
 *     of hair_render_async serves no other call until hair_ws_finish.
 *   - a HIP runtime error makes the call return HAIR_EDEVICE and poisons the context: every
 *     later call on it fails with HAIR_EDEVICE.
 */
#ifndef HAIR_H
#define HAIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HAIR_OK 0
#define HAIR_EINVAL (-1)   /* bad shape, non-finite value, out-of-range argument */
#define HAIR_ENOMEM (-2)   /* the HBM budget (or the device) cannot hold the request */
#define HAIR_ENOENT (-3)   /* unknown asset or level */
#define HAIR_EDEVICE (-4)  /* no usable device or a HIP error (context poisoned) */
#define HAIR_ERANGE (-5)   /* the frame exceeds a fixed capacity (see hair_stats) */

#define HAIR_MAX_LIGHTS 8

typedef struct hair_ctx hair_ctx;
typedef struct hair_ws hair_ws;

/* Single-fibre scattering model of a material. */
#define HAIR_MODEL_RTTRT 0 /* near-field R / TT / TRT; attenuation from eta and sigma_a */
#define HAIR_MODEL_RTTD 1  /* R / TT / D with constant RGB attenuations (Sec. 3.1, eq. bcsdf) */

/* Fibre material.
 * model HAIR_MODEL_RTTRT reads: relative index eta (> 1), longitudinal shift alpha (radians,
 *   |alpha| <= 0.5; R lobe, TT and TRT use -alpha/2 and -3 alpha/2), longitudinal width beta_m
 *   (radians, in (0, 2), standard deviation of theta_h for R; TT and TRT use beta_m/2 and
 *   2 beta_m), azimuthal width beta_n (radians, in (0, 4), standard deviation); the per-strand
 *   absorption sigma_a sets the attenuations.
 * model HAIR_MODEL_RTTD reads (Sec. 3.1 and the lobe shapes of Sec. 4; Sec. 6 gives the
 *   ranges 0.08-0.15, 0.12-0.3, 0.2-0.4 and the attenuations): beta_r, beta_tt (radians, in
 *   (0, 2): M_R = 1/2 G(beta_r, theta_h), M_TT = 1/2 G(beta_tt, theta_h)), gamma_tt (radians,
 *   in (0, 4): N_TT = G(gamma_tt, phi - pi)), a_r, a_tt, a_d (RGB, >= 0, a_r + a_tt + a_d <= 1
 *   per channel); M_D = 1/pi and N_R = N_D = 1/(2 pi).  sigma_a is not used.
 * Fields the chosen model does not read are ignored. */
typedef struct hair_material {
    float eta, alpha, beta_m, beta_n;
    int32_t model;
    float beta_r, beta_tt, gamma_tt;
    float a_r[3], a_tt[3], a_d[3];
} hair_material;

/* Pinhole camera.  rot: row-major world->view rotation; the view looks along -z with +y up.
 * Pixel (i, j) has its centre at (i + 0.5, j + 0.5) with x right and y down:
 * x = cx + fx * vx / (-vz), y = cy - fy * vy / (-vz).  Points nearer than z_near are culled. */
typedef struct hair_camera {
    float pos[3];
    float rot[9];
    float fx, fy, cx, cy;
    int32_t width, height;
    float z_near;
} hair_camera;

/* kind 0: directional, vec = unit direction toward the light, rgb = irradiance E.
 * kind 1: point, vec = position (m), rgb = intensity I (E = I / distance^2). */
typedef struct hair_light {
    int32_t kind;
    float vec[3];
    float rgb[3];
} hair_light;

/* Filled by hair_render when non-NULL (the call then synchronises its stream). */
typedef struct hair_stats {
    uint64_t fragments;          /* accepted (segment, pixel) fragments */
    uint64_t pairs;              /* (tile, segment) binning pairs */
    uint32_t segments;           /* rows drawn: the level's segments, or with long segments as pieces */
    uint32_t segments_visible;   /* after near-plane, guard-band and size culling */
    uint32_t segments_culled_long; /* culled as too long (more than 64 pieces of 1000 px, or any
                                      segment beyond 1024 px in hair_render_noalloc) or wider
                                      than 2048 px in half-width */
    uint32_t overflow_pixels;    /* pixels that could not be ordered (none in a forward frame; backward: > 64 slices) */
    float ms_total;              /* GPU time of the call's kernels (hipEvent) */
    float ms_project;            /* of which before shading: projection, binning, coverage, emission */
    float ms_bin;                /* 0: binning is timed within ms_project */
    float ms_tile;               /* of which the shading pass (sort, shade, blend) */
    uint32_t deep_pixels;        /* pixels deeper than one LDS batch, rendered in depth-key slices */
    uint32_t batches;            /* LDS batches of the frame */
} hair_stats;

#define HAIR_PIXEL_CAPACITY 1536   /* fragments per LDS batch */
#define HAIR_TILE 16               /* tile edge (pixels) */

/* Library version (major * 10000 + minor * 100 + patch). */
int hair_version(void);

/* Thread-local description of the last failure on the calling thread. */
const char* hair_last_error(void);

/* Number of HIP devices (0 when none); never fails. */
int hair_device_count(void);

/* Create a context on HIP device `device` with an HBM budget in bytes (0 = 90% of the
 * device's memory).  device = -1 makes a host-only context: every call validates its
 * arguments and then returns HAIR_EDEVICE without touching a device (used to test argument
 * checking on machines without a GPU).  *out receives the context. */
int hair_ctx_create(int32_t device, uint64_t hbm_budget_bytes, hair_ctx** out);
/* Frees the context's assets and its default workspace; workspaces made by hair_ws_create
 * must be destroyed before their context. */
int hair_ctx_destroy(hair_ctx* ctx);
/* Bytes the context holds and its budget. */
int hair_ctx_memory(hair_ctx* ctx, uint64_t* used_bytes, uint64_t* budget_bytes);

/* A render workspace: per-call scratch (segment records, tile lists) that grows on demand up
 * to max_bytes (0 = no limit beyond the context budget).  One workspace per concurrent
 * render stream. */
int hair_ws_create(hair_ctx* ctx, uint64_t max_bytes, hair_ws** out);
int hair_ws_destroy(hair_ws* ws);
/* Bytes the workspace holds on the device now and its limit (0 = none). */
int hair_ws_memory(hair_ws* ws, uint64_t* held_bytes, uint64_t* max_bytes);
/* Change the workspace's limit (0 = none) for its later calls; buffers it already holds are
 * kept, so held bytes may exceed a lowered limit until hair_ws_trim.  A call that would grow
 * the workspace beyond the limit fails with HAIR_ENOMEM. */
int hair_ws_set_limit(hair_ws* ws, uint64_t max_bytes);
/* Free every buffer the workspace holds (its next frame sizes them afresh, as a first frame
 * does).  HAIR_EINVAL while it holds a frame of hair_render_async. */
int hair_ws_trim(hair_ws* ws);
/* Bytes a render of n_segments at width x height needs in a workspace (upper bound used
 * for admission control); pairs_estimate = expected (tile, segment) pairs (0 = 4 per segment). */
uint64_t hair_ws_estimate(int64_t n_segments, int32_t width, int32_t height, int64_t pairs_estimate);

/* Upload a strand asset (Sec. 5.1 input: strand polylines, per-strand width and absorption).
 *   xyz_soa     host float[3][n_strands * verts_per_strand]: x row, y row, z row (metres);
 *               vertex k of strand s at column s * verts_per_strand + k.
 *   width       host float[n_strands]: fibre diameter (m), > 0.
 *   sigma_a_soa host float[3][n_strands]: absorption per unit fibre radius (RGB), >= 0.
 *   material    host, see hair_material (ranges there; out of range -> HAIR_EINVAL).
 * verts_per_strand >= 2.  All values finite.  *asset_out receives the asset id; level 0 is
 * the strands.  Data stays resident in HBM until hair_release or hair_ctx_destroy. */
int hair_upload(hair_ctx* ctx, int32_t n_strands, int32_t verts_per_strand,
                const float* xyz_soa, const float* width, const float* sigma_a_soa,
                const hair_material* material, void* stream, int32_t* asset_out);
int hair_release(hair_ctx* ctx, int32_t asset);

/* Build thick-hair levels 1..n_levels from cluster assignments (Sec. 5.1 steps 2-3), on the
 * device.  n_clusters host int[n_levels] (finer -> coarser); assign host int[n_levels][n_strands]
 * with values in [0, n_clusters[l]), every cluster non-empty.  Per level and cluster:
 * centre polyline = member mean of each vertex (float64 sums in member order); per segment
 * the 2x2 covariance of member midpoints orthogonal to the centre tangent gives the ellipse
 * (semi-axis = r + 2 sqrt(eigenvalue), a^ = major direction); n_total = member count,
 * sigma_a = member mean, r = mean width / 2.  Replaces any existing levels. */
int hair_build_lod(hair_ctx* ctx, int32_t asset, int32_t n_levels, const int32_t* n_clusters,
                   const int32_t* assign, void* stream);

/* Level count (not counting level 0), clusters per level (host int[n_levels + 1], entry 0 =
 * strands) and segments per strand. */
int hair_lod_info(hair_ctx* ctx, int32_t asset, int32_t* n_levels, int32_t* counts, int32_t max_counts,
                  int32_t* segs_per_strand);

/* Export (get) or import (set) a thick-hair level as host arrays (the stored configuration
 * of Sec. 6, "Memory cost and initialization time").  K clusters, S segments per centre line:
 *   centers float[K][S+1][3], ahat float[K][S][3], axes float[K][S][2] (|a|, |b|),
 *   n_total int[K], sigma_a float[3][K], r float[K].
 * set: level in 1..n_levels+1 (n_levels+1 appends); get: level in 1..n_levels.  Replacing a
 * level by one with the same cluster count keeps the clusters' memberships from
 * hair_build_lod (cluster c stays cluster c, so per-group LoD stays available); appending a
 * level or changing its cluster count drops the nested hierarchy. */
int hair_get_lod(hair_ctx* ctx, int32_t asset, int32_t level, int32_t n_clusters,
                 float* centers, float* ahat, float* axes, int32_t* n_total, float* sigma_a, float* r);
int hair_set_lod(hair_ctx* ctx, int32_t asset, int32_t level, int32_t n_clusters,
                 const float* centers, const float* ahat, const float* axes, const int32_t* n_total,
                 const float* sigma_a, const float* r, void* stream);

/* Overwrite a level's fitted parameters from device arrays (LoD fitting):
 * axes float[K][S][2] (> 0), r float[K] (> 0), sigma_a float[3][K] (>= 0); any may be NULL
 * to keep it.  Enqueued on `stream` (ordered with renders on the same stream). */
int hair_set_cluster_params(hair_ctx* ctx, int32_t asset, int32_t level, const float* axes,
                            const float* r, const float* sigma_a, void* stream);

/* Per-request level choice (Sec. 5.1 step 5 with eps_w of Sec. 6): the coarsest level whose
 * widest visible thick hair (2 * half-width, pixels) is <= eps_w_px; 0 when none is.
 * Synchronises `stream`.  ws: scratch (NULL = a context-owned one). */
int hair_select_level(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam,
                      float eps_w_px, void* stream, int32_t* level_out);

/* Deep opacity map shadows (Sec. 5.2, shadow pass; the count of hairs a light path crosses
 * scales and widens the forward lobes as in Sec. 4).  Every directional light gets a map of
 * resolution x resolution texels over the hair seen along it and `layers` depth layers of
 * layer_depth (world units) from each texel's first hair; a fragment's count of hairs in front
 * (one layer of bias, linear in depth, bilinear across texels) is added to its forward count:
 * strands are shaded by the aggregated model with one hair and n_F = 1 + count.  Point lights
 * are not shadowed.  resolution in [16, 4096], layers in [1, 7], layer_depth > 0. */
typedef struct hair_shadow {
    int32_t resolution;
    int32_t layers;
    float layer_depth;
} hair_shadow;

/* Render one frame (the hot path: projection and half-width, Sec. 5.2; binning and coverage
 * of the strips; per fragment f_single (Sec. 3.1, eq. bcsdf) or f_ours (Sec. 4, eq. our_bcsdf)
 * times E cos(theta_i) (Sec. 3); front-to-back compositing in (depth key, segment id) order).
 * rgba_out: device float[height][width][4], premultiplied
 * (C, 1 - T) over transparent black, written in full.  n_lights in 1..HAIR_MAX_LIGHTS.
 * The call synchronises `stream` once, at the end.  The first frame on a workspace (and a
 * frame that outgrows the workspace's buffers, which is then rendered again) also
 * synchronises twice in between to size them, with a quarter of headroom kept for the
 * frames that follow.  Pixels of any depth are rendered exactly, in slices of at most
 * HAIR_PIXEL_CAPACITY fragments cut by depth key and, inside a key shared by more fragments,
 * by segment id. */
int hair_render(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                const hair_light* lights, int32_t n_lights, float* rgba_out, void* stream,
                hair_stats* stats);

/* The frame of hair_render (same operation, same output, same errors) for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The call allocates nothing (no hipMalloc, hipFree, pinned host memory or
 * event creation): its scratch buffers are carved, per frame and at their exact sizes, from a
 * static device array of hair_noalloc_scratch_bytes() bytes (64 MiB) that every device the
 * library runs on holds until the process ends; the context set it up when it was created.
 * A frame needing more returns HAIR_ENOMEM before the image is written (e.g. 1,000 strands x
 * 16 segments at 256 x 256 needs about 4 MB; a 1920 x 1080 frame of 100k x 32 strands does not
 * fit).  Inputs (the resident asset) and the output (device float[height][width][4],
 * caller-owned) are as for hair_render.  The frame is sized on the device, read back twice
 * and synchronised at its end, as a first hair_render on a workspace.  Every call on one
 * device shares that device's scratch, which keeps the last call's contents: calls on one
 * context are serialised, but calls that overlap on one device from different contexts race
 * and must not be made. */
int hair_render_noalloc(hair_ctx* ctx, int32_t asset, int32_t level, const hair_camera* cam,
                        const hair_light* lights, int32_t n_lights, float* rgba_out, void* stream,
                        hair_stats* stats);
/* Size in bytes of the static scratch of hair_render_noalloc. */
uint64_t hair_noalloc_scratch_bytes(void);

/* The same frame as hair_render (same operation, same output) without waiting for it: on a
 * workspace that has rendered before (its buffer capacities are known) the frame is enqueued
 * on `stream` and the call returns at once, so that a caller can keep frames in flight (one
 * per workspace) with no host round trip between them.  On a workspace without capacities
 * the frame runs synchronously, as hair_render.  ws is required; the workspace then holds
 * the frame until hair_ws_finish, and every other call on it fails with HAIR_EINVAL until
 * then.  cam and lights are copied; rgba_out must stay valid until the frame is finished.
 * Argument errors are reported here, frame errors by hair_ws_finish. */
int hair_render_async(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                      const hair_light* lights, int32_t n_lights, float* rgba_out, void* stream);

/* Waits for the workspace's frame of hair_render_async and checks it as hair_render does: a
 * frame that outgrew the workspace's buffers is rendered again, synchronously, on its stream.
 * Fills stats (may be NULL) and returns the frame's status (HAIR_ERANGE as for hair_render).
 * With no frame held: HAIR_OK and zeroed stats. */
int hair_ws_finish(hair_ws* ws, hair_stats* stats);

/* hair_render with deep opacity map shadows (see hair_shadow) at a strand or thick-hair level
 * (mixed frames: hair_render_mixed_shadowed).  One shadow pass per directional light runs on `stream`
 * before the frame (sized like a frame, see hair_render); stats describe the
 * camera frame, with ms_total including the shadow passes.  The workspace keeps the maps
 * until its next shadowed render. */
int hair_render_shadowed(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                         const hair_light* lights, int32_t n_lights, const hair_shadow* shadow, float* rgba_out,
                         void* stream, hair_stats* stats);

/* hair_render_mixed with deep opacity map shadows (see hair_shadow): the shadow pass of every
 * directional light rasterises the frame's own rows (each (g, k) at its level: strands with
 * their radius, thick hairs with their cross-section and hair count), and each strand or
 * thick-hair fragment adds the hairs in front of it to its forward count as in
 * hair_render_shadowed.  Same levels, deferred update, output and errors as hair_render_mixed;
 * stats->ms_total includes the shadow passes. */
int hair_render_mixed_shadowed(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam,
                               const hair_light* lights, int32_t n_lights, int32_t* levels, float eps_w_px,
                               const hair_shadow* shadow, float* rgba_out, void* stream, hair_stats* stats);

/* hair_render at a thick-hair level (level >= 1) with curved centre lines (Sec. 5.2: the
 * tessellation stage subdivides each thick hair by its distance to the camera; Sec. 6: spline
 * centre lines).  Each centre line is the uniform Catmull-Rom spline through the level's centre
 * vertices (ends clamped); segment k is split into m equal parameter steps, m the smallest
 * integer in [1, max_sub] with 16 * m * max_px >= its snapped screen length in 1/16 pixels
 * (segments with an endpoint off screen are not split).  A step keeps its segment's
 * cross-section, hair count, radius and absorption.  max_px in [1, 4096], max_sub in [1, 16];
 * synchronises `stream` once more than hair_render; stats->segments counts the steps. */
int hair_render_curved(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                       const hair_light* lights, int32_t n_lights, int32_t max_px, int32_t max_sub, float* rgba_out,
                       void* stream, hair_stats* stats);

/* Per-group, per-segment LoD (Sec. 5.1 step 5; Sec. 5.2 "Dynamic LoD selection",
 * eq. lod_select).  Available when hair_build_lod built 1..7 levels that nest: every cluster
 * of a finer level lies inside one cluster of the coarsest level.  Those coarsest clusters
 * are the G groups; a frame chooses a level L(g, k) in 0..n_levels (0 = the strands) for every
 * group g and segment index k and renders, for each (g, k), the k-th segments of the level's
 * owners (strands or clusters) inside g.  levels: device int32[G][S] (caller-owned).
 * The width of (g, k) at level l is the largest 2 * half-width (pixels) over those segments
 * that are visible (0 when none is).
 * hair_lod_groups: G, or HAIR_EINVAL when the asset has no nested hierarchy. */
int hair_lod_groups(hair_ctx* ctx, int32_t asset, int32_t* n_groups);

/* Initial levels: for every (g, k) the coarsest level l >= 1 whose width is <= eps_w_px,
 * else 0.  Writes levels; synchronises `stream`. */
int hair_lod_init(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam,
                  float eps_w_px, int32_t* levels, void* stream);

/* Render one frame at the per-(g, k) levels (mixed strands and thick hairs, each shaded by
 * its own model); same output, synchronisation and errors as hair_render (HAIR_EINVAL when a
 * levels entry lies outside [0, n_levels]; stats->segments counts the rendered segments).
 * With eps_w_px > 0 the levels are then updated in place for the next frame (deferred
 * selection): with w the width at the frame's level L and w_c the width one level coarser,
 * L - 1 (not below 0) if w > eps_w_px, L + 1 if L < n_levels and w_c <= eps_w_px, else L.
 * eps_w_px <= 0 leaves levels unchanged. */
int hair_render_mixed(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam,
                      const hair_light* lights, int32_t n_lights, int32_t* levels, float eps_w_px,
                      float* rgba_out, void* stream, hair_stats* stats);

/* Vector-Jacobian product of hair_render at a thick-hair level (level >= 1) with respect to
 * the level's fitted parameters (Sec. 4: the aggregated model's |a|, |b| per cluster segment,
 * r and sigma_a per cluster; the half-width of Sec. 5.2 follows |a|, |b|).  Pixels deeper
 * than one LDS batch are differentiated slice by slice in (key, segment id) order (HAIR_ERANGE
 * only for a pixel needing more than 64 slices of HAIR_PIXEL_CAPACITY fragments): given
 * d_rgba (device float[height][width][4]) writes
 *   d_axes    device float[K][S][2]  d/d|a|, d/d|b|
 *   d_r       device float[K]        d/dr
 *   d_sigma_a device float[3][K]     d/dsigma_a
 * of sum(d_rgba * rgba) (overwritten).  The fragment set is recomputed, not stored, and held
 * fixed (coverage is piecewise constant in the parameters). */
int hair_render_backward(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level,
                         const hair_camera* cam, const hair_light* lights, int32_t n_lights,
                         const float* d_rgba, float* d_axes, float* d_r, float* d_sigma_a,
                         void* stream);

/* Measurement export: the device's issue rate of one instruction kind, in lane-operations per
 * second, from a kernel of independent chains at full occupancy (256 x 32 blocks of 256
 * threads, iters rounds of 8 operations per thread) timed with hipEvents on the legacy default
 * stream.  kind 0: v_fma_f32, 1: v_exp_f32, 2: v_rcp_f32, 3: v_sqrt_f32, 4: v_mul_lo_u32,
 * 5: v_mul_u32_u24.  Uses the context's static scratch (see hair_render_noalloc). */
int hair_debug_issue_rate(hair_ctx* ctx, int32_t kind, int32_t iters, double* ops_per_s);

/* Test exports of the last hair_render on `ws` (synchronise and copy to host):
 * segments: int[n][6] (XA, YA, XB, YB, hw_fx, flags: bit0 visible, bit1 negative h side,
 *           bit2 culled for size, bit3 thick hair of a mixed frame) and float[n][3]
 *           (izA, izB, hw px).
 * bins:     tile_start uint[n_tiles + 1], tile_segs uint[pairs] (each tile's segment ids,
 *           in no particular order). */
int hair_debug_segments(hair_ws* ws, int64_t n, int32_t* rec_i, float* rec_f);
int hair_debug_bins(hair_ws* ws, int64_t n_tiles, uint32_t* tile_start, int64_t n_pairs, uint32_t* tile_segs);

/* Test export of the shadow map of light `light` from the last hair_render_shadowed on `ws`:
 * texels host float[R * R][8] = (iz0, C_0 .. C_6) per texel, row-major (iz0: z_ref minus the
 * depth of the texel's first hair along the light, 0 when the texel holds no hair; C_k: hairs
 * counted through layer k; entries beyond the layer count repeat the last layer's total),
 * grid host float[16] = (e1, e2, d, omega, u0, v0, texel size, z_ref).
 * HAIR_EINVAL when that light had no map. */
int hair_debug_dom(hair_ws* ws, int32_t light, float* texels, float* grid);

/* Test export of composited fragment lists: renders like hair_render and, for pixels in
 * [x0, x0 + w) x [y0, y0 + h), writes per pixel its fragment count (host uint[h][w]) and
 * its fragments in compositing order (host arrays of cap entries, pixels row-major):
 * key uint, segment id uint, alpha float, offset h float.  A pixel's dump holds at most
 * max(HAIR_PIXEL_CAPACITY, cap / (w h)) fragments (device scratch of that many entries per
 * pixel).  HAIR_ERANGE if cap or a pixel's room is short, or if a pixel of the frame exceeded
 * the capacity at one depth key. */
int hair_debug_fragments(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level,
                         const hair_camera* cam, const hair_light* lights, int32_t n_lights,
                         int32_t x0, int32_t y0, int32_t w, int32_t h, uint32_t* counts,
                         int64_t cap, uint32_t* keys, uint32_t* segs, float* alpha, float* hoff,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HAIR_H */
