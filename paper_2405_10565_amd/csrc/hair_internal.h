// Internal types shared by the library's HIP sources (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hair.h"

namespace hair {

constexpr int kTile = HAIR_TILE;                 // tile edge in pixels
constexpr int kTilePix = kTile * kTile;          // pixels per tile = threads per tile block
constexpr int kCap = HAIR_PIXEL_CAPACITY;        // fragments per LDS batch
constexpr int kGuard = 16384;                    // guard band, 1/16-px units (1024 px)
constexpr int kMaxAxis = 16384;                  // longest segment (or piece) extent per axis (1/16 px)
constexpr int kMaxHwFx = 32768;                  // widest coverage half-width (1/16 px)
constexpr int kSplitLen = 16000;                 // a longer segment is drawn as pieces of at most this extent
constexpr int kMaxPieces = 64;                   // pieces per segment (row = segment << 6 | piece)
constexpr int kMaxListLen = (1 << 24) - 1;       // per-tile list limit (24-bit local index)
constexpr int kBinThreads = 512;                 // threads per binning block
constexpr int kMaxLdsTiles = 36864;              // per-tile LDS counters of one binning pass (144 KiB)

// Projected segment, one per segment of the rendered level (32 bytes, AoS for gathers).
struct alignas(16) SegRec {
    int32_t xa, ya, xb, yb;   // endpoints, 1/16-pixel units
    int32_t hwfx;             // coverage half-width ceil(16 hw) in bits 0..15; flags above
    float iza, izb;           // inverse view depth at the endpoints
    float hw;                 // half-width in pixels
};
// Per-segment shading inputs gathered once per frame by k_project (64 bytes, one aligned
// half cache line per fragment instead of five scattered reads):
//   q0 = (pA, sigma_r)  q1 = (pB, sigma_g)  q2 = (a^, sigma_b)  q3 = (|a|, |b|, n_total, r)
// (strands in mixed frames leave a^ and q3 unused).  In a strand-level frame the same 64 bytes
// hold the packed strand layout of pack_strand_shade instead, which also carries the screen
// record's fields the shading needs, so that a fragment's gather is one line.
struct ShadeRec {
    float4 q0, q1, q2, q3;
};
static_assert(sizeof(SegRec) == 32 && sizeof(ShadeRec) == 64, "records are stored as 16-byte words");

constexpr int32_t kFlagVisible = 1 << 16;
constexpr int32_t kFlagNegSide = 1 << 17;        // h > 0 lies on the e x d < 0 side
constexpr int32_t kFlagCulledLong = 1 << 18;
constexpr int32_t kFlagThick = 1 << 19;          // mixed frames: a thick-hair segment
constexpr int32_t kFlagSplit = 1 << 20;          // culled as longer than kMaxAxis, both endpoints on the guard band
constexpr int32_t kHwMask = 0xFFFF;

struct CamConst {
    float pos[3];
    float rot[9];
    float fx, fy, cx, cy, z_near;
    int32_t W, H;
};

struct LightConst {
    int32_t kind;
    float vec[3];
    float rgb[3];
};

// Deep opacity map of one directional light.  The frame (e1, e2 across the light, d = -omega
// along it) is set on the host; the grid origin and texel size are found on the device from
// the level's bounds (k_dom_grid) and read from device memory by the later kernels.
struct DomBasis {
    float e1[3], e2[3], d[3], omega[3];
};
struct DomGrid {
    DomBasis b;
    float u0, v0, s, k16, z_ref;    // texel (i, j) covers u0 + s [i, i+1) x v0 + s [j, j+1)
    int32_t R;
};
constexpr int kDomMaxLayers = 7;
// What shading reads per light; grid == nullptr: unshadowed.
struct DomView {
    const DomGrid* grid;
    const float4* tex;              // [R * R][2]: (iz0, C_0, C_1, C_2), (C_3 .. C_6); iz0 = 0: no hair
    int32_t K;
    float delta;                    // layer depth (world units)
};

struct LightsConst {
    int32_t n;
    LightConst l[HAIR_MAX_LIGHTS];
    DomView dom[HAIR_MAX_LIGHTS];
};

// Material constants derived on the host from hair_material (Sec. 6 parameters).
struct MatConst {
    float eta;
    float inv_eta2;          // 1 / eta^2
    float alpha_p[3];        // longitudinal shifts of R, TT, TRT
    float beta_p[3];         // longitudinal standard deviations of R, TT, TRT
    float g_amp[3];          // M_p = g_amp exp(-g_k x^2): 1 / (2 beta_p sqrt(2 pi))
    float g_k[3];            //                            1 / (2 beta_p^2)
    float g_k2[3];           // g_k log2(e)
    float beta_n;            // azimuthal standard deviation
    float s;                 // logistic scale sqrt(3) beta_n / pi
    float inv_s;             // 1 / s
    float inv_s_l2;          // log2(e) / s
    float n_norm;            // trimmed-logistic normaliser 1 / (s tanh(pi / 2s))
    float mn_amp[3];         // g_amp[p] n_norm: the amplitude of M_p N_p
    float cdf_lo, cdf_scale; // trimmed CDF: (sigmoid(x / s) - cdf_lo) * cdf_scale on [-pi, pi]
    // R / TT / D model (model == 1); the fields above serve model 0
    int32_t model;
    float d_amp[2];          // M_R, M_TT = d_amp exp2(-d_k2 theta_h^2): 1 / (2 beta sqrt(2 pi))
    float d_k2[2];           //                                     log2(e) / (2 beta^2)
    float d_beta2[2];        // beta_R^2, beta_TT^2
    float n_amp, n_k2;       // N_TT = n_amp exp2(-n_k2 psi^2): 1 / (gamma sqrt(2 pi)), log2(e) / (2 gamma^2)
    float gamma2;            // gamma_TT^2
    float A[3][3];           // [R, TT, D][channel] attenuations
    float aF[3], aB[3];      // front / back hemisphere albedos
    float var_f, var_b;      // attenuation-weighted longitudinal variances (front / back)
};

// One renderable level, device pointers.
struct LevelDev {
    int32_t kind;            // 0 = strands, 1 = thick hairs
    int32_t nseg;            // segments in the level
    int32_t S;               // segments per strand / centre line
    int32_t n_owner;         // strands or clusters (stride of the SoA per-owner arrays)
    const float* vx;         // vertex SoA [n_owner * (S + 1)]
    const float* vy;
    const float* vz;
    const float* width;      // strands: diameter [n_owner]
    const float* sig;        // absorption SoA [3][n_owner]
    const float* ahat;       // thick hairs: major axis direction SoA [3][nseg]
    const float* axes;       // thick hairs: (|a|, |b|) [nseg][2]
    const int32_t* n_total;  // thick hairs: member count [n_owner]
    const float* r;          // thick hairs: hair radius [n_owner]
};

// A nested LoD hierarchy for per-group, per-segment level choice: levels 0 (strands) ..
// n_levels (coarsest), groups = clusters of the coarsest level, and each level's owners listed
// by group (grp_owner[l][grp_start[l][g] .. grp_start[l][g + 1]), ascending owner ids).
constexpr int kMaxMixedLevels = 7;               // cluster levels a mixed frame may use
struct HierDev {
    int32_t n_levels, G, S;
    LevelDev lv[kMaxMixedLevels + 1];
    const int32_t* grp_start[kMaxMixedLevels + 1];
    const int32_t* grp_owner[kMaxMixedLevels + 1];
};

// Global counters a render accumulates (zeroed at the start of each call).
struct Counters {
    unsigned long long fragments;
    uint32_t visible;
    uint32_t culled_long;
    uint32_t overflow_pixels;
    uint32_t max_hw_bits;    // float bits of the largest visible half-width (non-negative)
    uint32_t list_overflow;  // tiles whose list exceeded the 24-bit local index
    uint32_t deep_pixels;    // pixels deeper than one LDS batch (rendered in depth-key slices)
    uint32_t cap_overflow;   // a frame size exceeded its buffer: the later passes did nothing
    uint32_t split_needed;   // segments culled as too long that pieces can draw (the frame is drawn again)
    uint32_t sizes[4];       // list entries, work items, fragments, batches of the frame
    uint32_t thick_batches;  // mixed frames: batches holding thick-hair fragments (listed in thick_list)
    unsigned long long phase[8];  // per-phase cycle sums (instrumented builds only)
};

// Buffer capacities a frame may fill without the host reading its sizes first.
struct FrameCaps {
    uint32_t pairs, items, frags, batches;
};

// Optional per-pixel fragment dump of a pixel rectangle (tests).
struct DebugDump {
    int32_t x0, y0, w, h;
    int32_t stride;          // entries per pixel
    uint32_t* counts;        // [h * w]
    uint32_t* keys;          // [h * w * stride]
    uint32_t* segs;
    float* alpha;
    float* hoff;
};

// Gradient outputs of the backward pass.
struct GradOut {
    const float* d_rgba;     // [H][W][4]
    float* d_axes;           // [nseg][2]
    float* d_r;              // [K]
    float* d_sig;            // [3][K]
    const uint32_t* rows;    // a frame of pieces: row -> segment << 6 | piece (nullptr: rows are segments)
};

// Device buffers of one frame's tile pipeline (T tiles of kTilePix pixels).
struct FrameBufs {
    int32_t T, ntx;
    const SegRec* seg;
    const ShadeRec* shade;
    const uint32_t* tile_start;   // [T + 1]: tile t's list is [tile_start[t], tile_start[t + 1])
    const uint32_t* list;         // segment ids
    const uint32_t* item_start;   // [T + 1] exclusive scan of per-tile work items
    const uint2* item_tab;        // [items] each work item's (tile, chunk of the tile's list)
    uint32_t* item_base;          // [items][kTilePix] each item's slice of each pixel's range
    uint32_t* pix_cnt;            // [T][kTilePix] fragments per pixel
    uint32_t* pix_kmin;           // [T][kTilePix] smallest depth key per pixel
    uint32_t* pix_kmax;           // [T][kTilePix] largest depth key per pixel
    uint32_t* pix_off;            // [T][kTilePix] exclusive prefix of pix_cnt within the tile
    uint8_t* pix_thick;           // [T][kTilePix] mixed frames: the pixel holds a thick-hair fragment
                                  // (nullptr in frames of one level)
    uint32_t* thick_list;         // [batches] mixed frames: table positions of the batches holding
                                  // thick-hair fragments (Counters::thick_batches of them)
    uint32_t* tile_tot;           // [T] fragments per tile
    uint32_t* tile_nb;            // [T] batches per tile
    uint32_t* batch_mask;         // [T][kTilePix / 32] pixels that start a batch
    const uint32_t* frag_base;    // [T + 1] exclusive scan of tile_tot
    const uint32_t* batch_start;  // [T + 1] exclusive scan of tile_nb
    uint4* batches;               // [batches]: packed (tile, p0, p1, oversized, first fragment, count), in launch order
    uint2* frags;                 // [fragments]: (depth key, segment | pixel << 24), see gid
    Counters* ctr;
    int32_t gid;                  // fragment records hold the global segment id (frames of fewer than
                                  // 2^24 rows, forward passes) instead of the index in the tile's list
};

// Kernel launchers (hair_kernels.hip).
hipError_t launch_project(const LevelDev& lv, const CamConst& cam, SegRec* seg, ShadeRec* shade, hipStream_t st);
// Exclusive scan of n counts into start[0..n] (start[n] = total); scratch holds
// 2 * ceil(n / 4096) + 2 words.
hipError_t launch_exscan(const uint32_t* cnt, uint32_t* start, int32_t n, uint32_t* scratch, hipStream_t st);
constexpr int kScanChunk = 4096;
inline size_t exscan_scratch_words(size_t n) { return 2 * ((n + kScanChunk - 1) / kScanChunk) + 2; }
// Binning blocks: nb blocks of kBinThreads own per_block consecutive segments each; tiles are
// counted in passes of `range` tiles.  The per-block count matrix M holds nb * T words.
struct BinPlan {
    int nb, per_block, range;
};
BinPlan bin_plan(int32_t nseg, int32_t T);
// M (nb * T words), blk (nb entries), tot (T words), tile_start (T + 1 words): per-block counts
// and segment statistics, tile totals and list offsets of the projected segments; ctr receives
// the visible / culled counts and the largest half-width.
hipError_t launch_bins(const SegRec* seg, int32_t nseg, const CamConst& cam, const BinPlan& p, uint32_t* M,
                       uint4* blk, uint32_t* tot, uint32_t* tile_start, Counters* ctr, uint32_t* scan_tmp,
                       hipStream_t st);
hipError_t launch_scatter(const SegRec* seg, int32_t nseg, const CamConst& cam, const BinPlan& p,
                          const uint32_t* tile_start, const uint32_t* M, uint32_t* list, const Counters* ctr,
                          hipStream_t st);
// Record the frame's sizes in ctr->sizes and flag ctr->cap_overflow when one exceeds its
// capacity (stage 1: list entries and work items; stage 2: fragments and batches).  Every
// later pass that would fill a sized buffer does nothing once the flag is set.
hipError_t launch_check_caps(const FrameBufs& f, const FrameCaps& caps, int stage, hipStream_t st);
hipError_t launch_tile_items(const uint32_t* tile_start, int T, uint32_t* items, hipStream_t st);
// Fused single-block forms for frames of at most kScanOneBlockTiles tiles: the items and their
// scan with the first capacity check; the fragment and batch offsets with the second.
constexpr int kScanOneBlockTiles = 1 << 16;
hipError_t launch_items_scan(const uint32_t* tile_start, int T, uint32_t* item_start, Counters* ctr,
                             uint32_t cap_pairs, uint32_t cap_items, hipStream_t st);
hipError_t launch_tile_scans(const FrameBufs& f, uint32_t* frag_base, uint32_t* batch_start, uint32_t cap_frags,
                             uint32_t cap_batches, hipStream_t st);
// Per-group LoD: initial levels, deferred update in place, and a mixed frame's selection
// (cnt and sel_start: G*S and G*S + 1 words; sel: one entry per selected segment).
hipError_t launch_lod_init(const HierDev& h, const CamConst& cam, float eps_w, int32_t* levels, hipStream_t st);
hipError_t launch_lod_update(const HierDev& h, const CamConst& cam, float eps_w, int32_t* levels, hipStream_t st);
hipError_t launch_select(const HierDev& h, const int32_t* levels, uint32_t* cnt, uint32_t* sel_start,
                         uint32_t* scan_tmp, hipStream_t st);
hipError_t launch_select_fill(const HierDev& h, const int32_t* levels, const uint32_t* sel_start, uint32_t* sel,
                              hipStream_t st);
hipError_t launch_project_mixed(const HierDev& h, const uint32_t* sel, int32_t nsel, const CamConst& cam, SegRec* seg,
                                ShadeRec* shade, hipStream_t st);
// grid: blocks to launch (>= the frame's work items / batches, read on the device)
hipError_t launch_count(const FrameBufs& f, const CamConst& cam, uint32_t grid, hipStream_t st);
hipError_t launch_tile_prep(const FrameBufs& f, hipStream_t st);
hipError_t launch_batch_records(const FrameBufs& f, hipStream_t st);
hipError_t launch_emit(const FrameBufs& f, const CamConst& cam, uint32_t grid, hipStream_t st);
hipError_t launch_batches(const FrameBufs& f, const LevelDev& lv, const CamConst& cam, const LightsConst& lights,
                          const MatConst& mat, uint32_t grid, float* rgba, const DebugDump* dbg, hipStream_t st);
hipError_t launch_batches_bwd(const FrameBufs& f, const LevelDev& lv, const CamConst& cam, const LightsConst& lights,
                              const MatConst& mat, uint32_t grid, const GradOut& grad, hipStream_t st);
hipError_t launch_build_centers(const float* vx, const float* vy, const float* vz, const float* width,
                                const float* sig, int32_t n_strands, int32_t V, const int32_t* members,
                                const int32_t* member_start, int32_t K, float* cx, float* cy, float* cz,
                                float* r, float* csig, int32_t* n_total, hipStream_t st);
hipError_t launch_build_ellipses(const float* vx, const float* vy, const float* vz, int32_t V,
                                 const int32_t* members, const int32_t* member_start, int32_t K,
                                 const float* cx, const float* cy, const float* cz, const float* r,
                                 float* ahat, float* axes, hipStream_t st);
// Curved thick hairs: per-segment steps cnt[nseg] and their exclusive scan start[nseg + 1]
// (scan_tmp: exscan scratch), the row list (g << 4 | j), and the rows' records.
hipError_t launch_tess(const LevelDev& lv, const CamConst& cam, int32_t max_px, int32_t max_sub, uint32_t* cnt,
                       uint32_t* start, uint32_t* scan_tmp, hipStream_t st);
hipError_t launch_tess_fill(const uint32_t* cnt, const uint32_t* start, int32_t nseg, uint32_t* rows, hipStream_t st);
hipError_t launch_split(const LevelDev& lv, const CamConst& cam, uint32_t* cnt, uint32_t* start, uint32_t* scan_tmp,
                        hipStream_t st);
hipError_t launch_split_mixed(const HierDev& h, const uint32_t* sel, int32_t nsel, const CamConst& cam, uint32_t* cnt,
                              uint32_t* start, uint32_t* scan_tmp, hipStream_t st);
hipError_t launch_project_split_mixed(const HierDev& h, const uint32_t* sel, const uint32_t* rows, int32_t nrows,
                                      const uint32_t* cnt, const CamConst& cam, SegRec* seg, ShadeRec* shade,
                                      hipStream_t st);
hipError_t launch_split_fill(const uint32_t* cnt, const uint32_t* start, int32_t nseg, uint32_t* rows, hipStream_t st);
hipError_t launch_project_split(const LevelDev& lv, const uint32_t* rows, int32_t nrows, const uint32_t* cnt,
                                const CamConst& cam, SegRec* seg, ShadeRec* shade, hipStream_t st);
hipError_t launch_project_tess(const LevelDev& lv, const uint32_t* rows, int32_t nrows, const uint32_t* cnt,
                               const CamConst& cam, SegRec* seg, ShadeRec* shade, hipStream_t st);
// Deep opacity map: the grid of one light from the level's bounds (part: 5 floats per bounds
// block, at most dom_bound_blocks(nseg) blocks), the light-view segment records, and the
// per-texel layers from the light view's fragment lists.
int dom_bound_blocks(int32_t nseg);
hipError_t launch_dom_grid(const LevelDev& lv, const ShadeRec* rows, const DomBasis& b, int32_t R, float* part, DomGrid* grid,
                           hipStream_t st);
hipError_t launch_project_light(const LevelDev& lv, const ShadeRec* rows, const DomGrid* grid, SegRec* seg,
                                hipStream_t st);
hipError_t launch_dom_resolve(const FrameBufs& f, const LevelDev& lv, const ShadeRec* rows, const DomGrid* grid, int32_t K, float delta,
                              int32_t R, uint32_t n_blocks, float4* tex, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
// The frame's per-pixel counters: n counts set to 0, key minima to ~0, key maxima to 0.
hipError_t launch_fill_pix(uint32_t* cnt, uint32_t* kmin, uint32_t* kmax, uint8_t* thick, size_t n, float* rgba,
                           size_t n_rgba4, const uint32_t* item_start, int T, uint2* item_tab, uint32_t cap_items,
                           hipStream_t st);   // also clears rgba (n_rgba4 pixels) when given
hipError_t launch_fill_f32(float* p, float v, size_t n, hipStream_t st);
hipError_t launch_probe_rate(int kind, int blocks, int iters, float* out, hipStream_t st);

}  // namespace hair
