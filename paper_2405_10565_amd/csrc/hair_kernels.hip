// Device kernels of the LoD hair renderer (gfx950 / MI355X).
//
// Frame pipeline, all on the caller's stream:
//   k_project        one thread per segment: float32 projection and 1/16-pixel snapping, screen
//                    half-width (Sec. 5.2, hair width calculation), culling.
//   k_bin_count      per block of consecutive segments: tile counts in LDS (no device atomics);
//   k_bin_offsets    column scan of the per-block count matrix -> each block's place in every list;
//   k_scan1          exclusive prefix sums (tile list offsets, work items, fragment and batch bases).
//   k_scatter        per block: append its segments' ids to the overlapped tiles' lists.
//   k_count          per (tile, list chunk): exact integer coverage -> per-pixel fragment counts
//                    (LDS-aggregated, then one global atomic per pixel).
//   k_tile_prep      per tile: pixel offsets, and whole pixels packed into batches of <= kCap.
//   k_emit           per (tile, list chunk): (key, local index) records into the fragment buffer
//                    and each pixel's depth-key range.
//   k_batch          one workgroup per batch, all in LDS: exact per-pixel order (bucket map over
//                    each pixel's key range, then each record's rank in its bucket), one lane per
//                    fragment for shading, front-to-back blending by a two-level segmented scan,
//                    coalesced RGBA stores.
// The integer-deciding steps (projection, snapping, half-width, depth key) are float32 with
// one rounding per operation and no contraction, so they match a float32 reference bit for bit.
#include <algorithm>

#include "hair_internal.h"
#include "hair_shading.h"
#include "hair_dual.h"

#pragma clang fp contract(off)

namespace hair {
namespace {

constexpr int kNT = 256;                   // threads per tile block (= pixels per tile)
constexpr int kPerThread = kCap / kNT;     // LDS batch fragments per thread
static_assert(kCap % kNT == 0, "a batch is kPerThread fragments per thread");

static_assert(kTile == 16, "the shifts below assume 16-pixel tiles in 1/16-pixel units");

__device__ inline int wave_max(int v) {
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// Inclusive prefix sum of x over the 64 lanes of a wave, in lane order, with DPP moves: shifts
// by 1, 2, 4 and 8 lanes inside each row of 16 (lanes shifted in from outside the row add 0),
// then the last lane of rows 0 and 2 added to rows 1 and 3, and lane 31 added to rows 2 and 3.
// (No LDS permutes: six adds with a moved operand.)
__device__ inline uint32_t wave_inclusive_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);   // row_bcast:15 -> rows 1, 3
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);   // row_bcast:31 -> rows 2, 3
    return x;
}

// Workgroups are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).  Map block b to
// work index w so that each XCD takes one contiguous range of work: neighbouring work units
// (batches of one tile, chunks of one list) then share that XCD's L2.
__device__ inline uint32_t xcd_contiguous(uint32_t b, uint32_t nb) {
    const uint32_t q = nb / 8, rem = nb % 8, x = b % 8, slot = b / 8;
    return x * q + min(x, rem) + slot;
}

// Its inverse on [0, nb): the block that xcd_contiguous sends to index r.
__device__ inline uint32_t xcd_block_of(uint32_t r, uint32_t nb) {
    const uint32_t q = nb / 8, rem = nb % 8, big = rem * (q + 1);
    uint32_t x, slot;
    if (r < big) {
        x = r / (q + 1);
        slot = r - x * (q + 1);
    } else {   // here q >= 1
        x = rem + (r - big) / q;
        slot = (r - big) - (x - rem) * q;
    }
    return slot * 8 + x;
}

// One LDS batch of the shading pass: tile, pixels [p0, p1), oversized (one pixel deeper than
// a batch), the frame-wide index of its first fragment and its fragment count.  The table is
// stored in launch order (record b is processed by block b, which keeps the tiles of an XCD
// contiguous), so a block reads its record without first reading the batch count.
struct BatchRec {
    int tile, p0, p1;
    bool over;
    uint32_t frag0, nfrag;
    bool thick;   // mixed frames: a pixel of the batch holds a thick-hair fragment
};
__device__ inline uint4 pack_batch(int tile, int p0, int p1, bool over, uint32_t frag0, uint32_t nfrag,
                                   bool thick = false) {
    return make_uint4((uint32_t)tile,
                      (uint32_t)p0 | ((uint32_t)p1 << 9) | (over ? 1u << 18 : 0u) | (thick ? 1u << 19 : 0u), frag0,
                      nfrag);
}
__device__ inline BatchRec unpack_batch(const uint4 r) {
    return BatchRec{(int)r.x, (int)(r.y & 511u), (int)((r.y >> 9) & 511u), ((r.y >> 18) & 1u) != 0, r.z, r.w,
                    ((r.y >> 19) & 1u) != 0};
}

// ---------------------------------------------------------------------------------------
// Projection (float32, fixed operation order).
struct PPoint {
    float X16, Y16, z, iz;
    bool ok;
};

__device__ inline PPoint project_point(const CamConst& c, float px, float py, float pz) {
    const float d0 = px - c.pos[0];
    const float d1 = py - c.pos[1];
    const float d2 = pz - c.pos[2];
    const float vx = (c.rot[0] * d0 + c.rot[1] * d1) + c.rot[2] * d2;
    const float vy = (c.rot[3] * d0 + c.rot[4] * d1) + c.rot[5] * d2;
    const float vz = (c.rot[6] * d0 + c.rot[7] * d1) + c.rot[8] * d2;
    PPoint p;
    p.z = -vz;
    const float xs = c.cx + c.fx * (vx / p.z);
    const float ys = c.cy - c.fy * (vy / p.z);
    p.iz = 1.0f / p.z;
    p.X16 = 16.0f * xs;
    p.Y16 = 16.0f * ys;
    p.ok = (p.z >= c.z_near) && (p.X16 >= -16384.0f) && (p.X16 <= (float)(16 * c.W + kGuard)) &&
           (p.Y16 >= -16384.0f) && (p.Y16 <= (float)(16 * c.H + kGuard));
    return p;
}

__device__ inline float norm3f(float x, float y, float z) { return sqrtf((x * x + y * y) + z * z); }
__device__ inline float dot_e(const float e[3], float x, float y, float z) { return (x * e[0] + y * e[1]) + z * e[2]; }

// Thick-hair half-width: support of the ellipse across the view at the segment midpoint.
__device__ inline float cluster_halfwidth(const CamConst& c, float ax, float ay, float az, float bx, float by,
                                          float bz, float zA, float zB, float hx, float hy, float hz, float a_len,
                                          float b_len) {
    const float tx = bx - ax, ty = by - ay, tz = bz - az;
    const float tl = norm3f(tx, ty, tz);
    const float ux = tx / tl, uy = ty / tl, uz = tz / tl;
    const float mx = (ax + bx) * 0.5f, my = (ay + by) * 0.5f, mz = (az + bz) * 0.5f;
    float wx = c.pos[0] - mx, wy = c.pos[1] - my, wz = c.pos[2] - mz;
    const float wl = norm3f(wx, wy, wz);
    wx = wx / wl;
    wy = wy / wl;
    wz = wz / wl;
    const float dwu = (wx * ux + wy * uy) + wz * uz;
    const float px = wx - dwu * ux, py = wy - dwu * uy, pz = wz - dwu * uz;
    const float pl = norm3f(px, py, pz);
    const float xx = px / pl, xy = py / pl, xz = pz / pl;
    const float yx = uy * xz - uz * xy, yy = uz * xx - ux * xz, yz = ux * xy - uy * xx;
    const float bhx = uy * hz - uz * hy, bhy = uz * hx - ux * hz, bhz = ux * hy - uy * hx;
    const float pa = a_len * ((hx * yx + hy * yy) + hz * yz);
    const float pb = b_len * ((bhx * yx + bhy * yy) + bhz * yz);
    float W = sqrtf(pa * pa + pb * pb);
    if (!(pl > 1e-7f)) W = fmaxf(a_len, b_len);
    const float zm = (zA + zB) * 0.5f;
    return (W * c.fy) / zm;
}

struct TileRect {
    int tx0, tx1, ty0, ty1;
};

// Tiles overlapped by the segment's integer box widened by its radius (x >> 8 = floor(x / 256),
// a 16-pixel tile in 1/16-pixel units; coordinates of a visible segment fit 32 bits).
__device__ inline TileRect tile_rect(const SegRec& s, int ntx, int nty) {
    const int R = (s.hwfx & kHwMask) + 8;
    const int lox = min(s.xa, s.xb) - R, hix = max(s.xa, s.xb) + R;
    const int loy = min(s.ya, s.yb) - R, hiy = max(s.ya, s.yb) + R;
    TileRect r;
    r.tx0 = max(lox >> 8, 0);
    r.tx1 = min(hix >> 8, ntx - 1);
    r.ty0 = max(loy >> 8, 0);
    r.ty1 = min(hiy >> 8, nty - 1);
    return r;
}

// The shading record of a strand segment in a strand-level frame: everything the shading pass
// reads for one fragment in one aligned 64-byte line (the screen record's coverage geometry,
// inverse depths and half-width, whose sign bit carries the side flag, then the world
// endpoints and the strand's absorption):
//   q0 = (xa, ya, xb, yb as int bits)  q1 = (iza, izb, +-hw, pA.x)  q2 = (pA.y, pA.z, pB.x, pB.y)
//   q3 = (pB.z, sigma_r, sigma_g, sigma_b)
__device__ inline void pack_strand_shade(const SegRec& r, float ax, float ay, float az, float bx, float by, float bz,
                                         float sr_, float sg_, float sb_, ShadeRec* sr) {
    const float shw = __uint_as_float(__float_as_uint(r.hw) | ((r.hwfx & kFlagNegSide) ? 0x80000000u : 0u));
    sr->q0 = make_float4(__int_as_float(r.xa), __int_as_float(r.ya), __int_as_float(r.xb), __int_as_float(r.yb));
    sr->q1 = make_float4(r.iza, r.izb, shw, ax);
    sr->q2 = make_float4(ay, az, bx, by);
    sr->q3 = make_float4(bz, sr_, sg_, sb_);
}

// Segment g of level lv, drawn between (ax, ay, az) and (bx, by, bz): its screen record
// (projection, snapping, half-width, culling, side of h > 0) and, when sr is given, its
// shading record (packed: the strand-level layout above; otherwise q0..q3 as ShadeRec states).
// The endpoints are the level's vertices, or points of a curved thick hair.
__device__ inline SegRec project_segment_at(const LevelDev& lv, int g, float ax, float ay, float az, float bx, float by,
                                            float bz, const CamConst& cam, ShadeRec* sr, bool packed = false) {
    const int owner = g / lv.S;
    const PPoint A = project_point(cam, ax, ay, az);
    const PPoint B = project_point(cam, bx, by, bz);
    if (sr && !packed) {   // whole float4 stores (q3 only for thick hairs)
        const float sb = lv.sig[2 * lv.n_owner + owner];
        float4 q2 = make_float4(0.f, 0.f, 0.f, sb);
        if (lv.kind != 0) q2 = make_float4(lv.ahat[g], lv.ahat[lv.nseg + g], lv.ahat[2 * lv.nseg + g], sb);
        sr->q0 = make_float4(ax, ay, az, lv.sig[owner]);
        sr->q1 = make_float4(bx, by, bz, lv.sig[lv.n_owner + owner]);
        sr->q2 = q2;
        if (lv.kind != 0)
            sr->q3 = make_float4(lv.axes[2 * g], lv.axes[2 * g + 1], (float)lv.n_total[owner], lv.r[owner]);
    }
    float hw;
    if (lv.kind == 0) {
        const float zm = (A.z + B.z) * 0.5f;
        hw = ((0.5f * lv.width[owner]) * cam.fy) / zm;
    } else {
        hw = cluster_halfwidth(cam, ax, ay, az, bx, by, bz, A.z, B.z, lv.ahat[g], lv.ahat[lv.nseg + g],
                               lv.ahat[2 * lv.nseg + g], lv.axes[2 * g], lv.axes[2 * g + 1]);
    }
    const float hw16 = 16.0f * hw;
    SegRec r;
    r.xa = r.ya = r.xb = r.yb = 0;
    r.hwfx = 0;
    r.iza = A.iz;
    r.izb = B.iz;
    r.hw = hw;
    if (A.ok && B.ok && isfinite(hw16) && hw16 >= 0.0f) {
        r.xa = (int)rintf(A.X16);
        r.ya = (int)rintf(A.Y16);
        r.xb = (int)rintf(B.X16);
        r.yb = (int)rintf(B.Y16);
        const float c16 = ceilf(hw16);
        const bool too_long = abs(r.xb - r.xa) > kMaxAxis || abs(r.yb - r.ya) > kMaxAxis;
        if (too_long || c16 > (float)kMaxHwFx) {
            // (a segment too long but not too wide is drawn again as pieces)
            r.hwfx = kFlagCulledLong | (too_long && c16 <= (float)kMaxHwFx ? kFlagSplit : 0);
        } else {
            r.hwfx = (int)c16 | kFlagVisible;
            // side of the screen normal (dY, -dX) on which h > 0 (toward y^ = u x x^)
            const float tx = bx - ax, ty = by - ay, tz = bz - az;
            const float tl = norm3f(tx, ty, tz);
            const float ux = tx / tl, uy = ty / tl, uz = tz / tl;
            const float mx = (ax + bx) * 0.5f, my = (ay + by) * 0.5f, mz = (az + bz) * 0.5f;
            float wx = cam.pos[0] - mx, wy = cam.pos[1] - my, wz = cam.pos[2] - mz;
            const float wl = norm3f(wx, wy, wz);
            wx /= wl; wy /= wl; wz /= wl;
            const float dwu = (wx * ux + wy * uy) + wz * uz;
            float px = wx - dwu * ux, py = wy - dwu * uy, pz = wz - dwu * uz;
            const float pl = fmaxf(norm3f(px, py, pz), 1e-30f);
            px /= pl; py /= pl; pz /= pl;
            const float yx = uy * pz - uz * py, yy = uz * px - ux * pz, yz = ux * py - uy * px;
            const float yvx = (cam.rot[0] * yx + cam.rot[1] * yy) + cam.rot[2] * yz;
            const float yvy = (cam.rot[3] * yx + cam.rot[4] * yy) + cam.rot[5] * yz;
            const float yvz = (cam.rot[6] * yx + cam.rot[7] * yy) + cam.rot[8] * yz;
            const float d0 = mx - cam.pos[0], d1 = my - cam.pos[1], d2 = mz - cam.pos[2];
            const float mvx = (cam.rot[0] * d0 + cam.rot[1] * d1) + cam.rot[2] * d2;
            const float mvy = (cam.rot[3] * d0 + cam.rot[4] * d1) + cam.rot[5] * d2;
            const float mvz = (cam.rot[6] * d0 + cam.rot[7] * d1) + cam.rot[8] * d2;
            const float Z = -mvz;
            const float sx = cam.fx * (yvx + (mvx / Z) * yvz);
            const float sy = -cam.fy * (yvy + (mvy / Z) * yvz);
            const float side = sx * (float)(r.yb - r.ya) - sy * (float)(r.xb - r.xa);
            if (side < 0.0f) r.hwfx |= kFlagNegSide;
        }
    }
    if (sr && packed)
        pack_strand_shade(r, ax, ay, az, bx, by, bz, lv.sig[owner], lv.sig[lv.n_owner + owner],
                          lv.sig[2 * lv.n_owner + owner], sr);
    return r;
}

__device__ inline SegRec project_segment(const LevelDev& lv, int g, const CamConst& cam, ShadeRec* sr,
                                         bool packed = false) {
    const int owner = g / lv.S, k = g - owner * lv.S;
    const int va = owner * (lv.S + 1) + k;
    return project_segment_at(lv, g, lv.vx[va], lv.vy[va], lv.vz[va], lv.vx[va + 1], lv.vy[va + 1], lv.vz[va + 1], cam,
                              sr, packed);
}

// A frame of one level: strand levels write the packed strand shading record.  The block's
// records are staged in LDS and stored as consecutive 16-byte words, so that every store
// instruction writes whole contiguous lines.
__global__ __launch_bounds__(256) void k_project(LevelDev lv, CamConst cam, SegRec* __restrict__ seg,
                                                 ShadeRec* __restrict__ shade) {
    __shared__ float4 s_seg[2 * 256];
    __shared__ float4 s_sh[4 * 256];
    const int t = threadIdx.x, g0 = blockIdx.x * 256, g = g0 + t;
    if (g < lv.nseg) {
        ShadeRec sr;
        sr.q3 = make_float4(0.f, 0.f, 0.f, 0.f);
        const SegRec r = project_segment(lv, g, cam, &sr, lv.kind == 0);
        s_seg[2 * t] = make_float4(__int_as_float(r.xa), __int_as_float(r.ya), __int_as_float(r.xb), __int_as_float(r.yb));
        s_seg[2 * t + 1] = make_float4(__int_as_float(r.hwfx), r.iza, r.izb, r.hw);
        s_sh[4 * t] = sr.q0;
        s_sh[4 * t + 1] = sr.q1;
        s_sh[4 * t + 2] = sr.q2;
        s_sh[4 * t + 3] = sr.q3;
    }
    __syncthreads();
    const int n = min(256, lv.nseg - g0);
    float4* dseg = reinterpret_cast<float4*>(seg + g0);
    for (int i = t; i < 2 * n; i += 256) dseg[i] = s_seg[i];
    float4* dsh = reinterpret_cast<float4*>(shade + g0);
    for (int i = t; i < 4 * n; i += 256) dsh[i] = s_sh[i];
}

// ---------------------------------------------------------------------------------------
// Per-group, per-segment LoD (Sec. 5.1 step 5; Sec. 5.2, eq. lod_select).  Groups are the
// clusters of the coarsest level; every finer level's owners (clusters, or strands at level
// 0) are listed per group in h.grp_owner[l] (CSR h.grp_start[l]).  The width of (g, k) at
// level l is the largest 2 hw over the visible k-th segments of level l's owners in g (0 if
// none is visible).  One wave per (g, k).

// Level of (g, k); levels outside [0, n_levels] are read as 0 (k_sel_count counts them in
// cnt[G S], which the caller zeroes and checks before rendering).
__device__ inline int level_at(const HierDev& h, const int32_t* levels, int gk) {
    const int L = levels[gk];
    return (L < 0 || L > h.n_levels) ? 0 : L;
}

// width bits of (g, k) at level l (non-negative float bits order like the floats)
__device__ inline uint32_t group_width_bits(const HierDev& h, int l, int g, int k, const CamConst& cam) {
    const LevelDev& lv = h.lv[l];
    const int b = h.grp_start[l][g], e = h.grp_start[l][g + 1];
    uint32_t w = 0;
    for (int i = b + (int)__lane_id(); i < e; i += 64) {
        const SegRec r = project_segment(lv, h.grp_owner[l][i] * lv.S + k, cam, nullptr);
        if (r.hwfx & kFlagVisible) w = max(w, __float_as_uint(2.0f * r.hw));
    }
    for (int off = 32; off >= 1; off >>= 1) w = max(w, (uint32_t)__shfl_xor((int)w, off));
    return w;
}

// Initial levels: the coarsest l >= 1 whose width is <= eps_w, else 0 (the strands).
__global__ __launch_bounds__(256) void k_lod_init(HierDev h, CamConst cam, float eps_w, int32_t* __restrict__ levels) {
    const int gk = (int)(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    if (gk >= h.G * h.S) return;
    const int g = gk / h.S, k = gk - g * h.S;
    int pick = 0;
    for (int l = h.n_levels; l >= 1; --l) {
        if (__uint_as_float(group_width_bits(h, l, g, k, cam)) <= eps_w) {
            pick = l;
            break;
        }
    }
    if (__lane_id() == 0) levels[gk] = pick;
}

// Deferred update from this frame's level L, with w_cur its width and w_c the width one
// level coarser: finer if w_cur > eps_w, coarser if w_c <= eps_w, else unchanged.
__global__ __launch_bounds__(256) void k_lod_update(HierDev h, CamConst cam, float eps_w, int32_t* __restrict__ levels) {
    const int gk = (int)(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    if (gk >= h.G * h.S) return;
    const int g = gk / h.S, k = gk - g * h.S;
    const int L = level_at(h, levels, gk);
    const float w_cur = __uint_as_float(group_width_bits(h, L, g, k, cam));
    int next = L;
    if (w_cur > eps_w) {
        next = max(L - 1, 0);
    } else if (L < h.n_levels) {
        const float w_c = __uint_as_float(group_width_bits(h, L + 1, g, k, cam));
        if (w_c <= eps_w) next = L + 1;
    }
    if (__lane_id() == 0) levels[gk] = next;
}

// Selection of a mixed frame: for every (g, k) the k-th segments of the owners of level
// L(g, k) in g, in (g, k, owner) order; entry = level << 28 | segment id of that level.
__global__ __launch_bounds__(256) void k_sel_count(HierDev h, const int32_t* __restrict__ levels,
                                                   uint32_t* __restrict__ cnt) {
    const int gk = blockIdx.x * blockDim.x + threadIdx.x;
    if (gk >= h.G * h.S) return;
    const int g = gk / h.S, raw = levels[gk], L = level_at(h, levels, gk);
    if (raw != L) atomicAdd(&cnt[h.G * h.S], 1u);
    cnt[gk] = (uint32_t)(h.grp_start[L][g + 1] - h.grp_start[L][g]);
}

__global__ __launch_bounds__(256) void k_sel_fill(HierDev h, const int32_t* __restrict__ levels,
                                                  const uint32_t* __restrict__ sel_start, uint32_t* __restrict__ sel) {
    const int gk = (int)(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    if (gk >= h.G * h.S) return;
    const int g = gk / h.S, k = gk - g * h.S, L = level_at(h, levels, gk);
    const int b = h.grp_start[L][g], e = h.grp_start[L][g + 1];
    const uint32_t o = sel_start[gk];
    for (int i = b + (int)__lane_id(); i < e; i += 64)
        sel[o + (uint32_t)(i - b)] = ((uint32_t)L << 28) | (uint32_t)(h.grp_owner[L][i] * h.S + k);
}

// (records staged in LDS and stored as consecutive 16-byte words, as in k_project)
__global__ __launch_bounds__(256) void k_project_mixed(HierDev h, const uint32_t* __restrict__ sel, int nsel,
                                                       CamConst cam, SegRec* __restrict__ seg,
                                                       ShadeRec* __restrict__ shade) {
    __shared__ float4 s_seg[2 * 256];
    __shared__ float4 s_sh[4 * 256];
    const int t = threadIdx.x, i0 = blockIdx.x * 256, i = i0 + t;
    if (i < nsel) {
        const uint32_t e = sel[i];
        const int L = (int)(e >> 28), g = (int)(e & 0x0FFFFFFFu);
        ShadeRec sr;
        sr.q3 = make_float4(0.f, 0.f, 0.f, 0.f);
        SegRec r = project_segment(h.lv[L], g, cam, &sr);
        if (h.lv[L].kind == 1) r.hwfx |= kFlagThick;
        // (a strand row's q3 is otherwise unused: its world radius, and -1 marking a strand, for
        // the shadow pass, which reads the rows' world data from these records)
        else sr.q3 = make_float4(0.5f * h.lv[L].width[g / h.lv[L].S], 0.0f, 0.0f, -1.0f);
        s_seg[2 * t] = make_float4(__int_as_float(r.xa), __int_as_float(r.ya), __int_as_float(r.xb), __int_as_float(r.yb));
        s_seg[2 * t + 1] = make_float4(__int_as_float(r.hwfx), r.iza, r.izb, r.hw);
        s_sh[4 * t] = sr.q0;
        s_sh[4 * t + 1] = sr.q1;
        s_sh[4 * t + 2] = sr.q2;
        s_sh[4 * t + 3] = sr.q3;
    }
    __syncthreads();
    const int n = min(256, nsel - i0);
    float4* dseg = reinterpret_cast<float4*>(seg + i0);
    for (int k = t; k < 2 * n; k += 256) dseg[k] = s_seg[k];
    float4* dsh = reinterpret_cast<float4*>(shade + i0);
    for (int k = t; k < 4 * n; k += 256) dsh[k] = s_sh[k];
}

// Exclusive scan of n counts by one 1024-thread block in coalesced chunks of 4096 (four
// consecutive counts per lane, wave shuffles, one LDS step across the 16 waves); start[n] =
// total.  For n up to kScanOneBlock.
constexpr int kScanOneBlock = 1 << 16;
__global__ __launch_bounds__(1024) void k_scan1(const uint32_t* __restrict__ cnt, uint32_t* __restrict__ start, int n) {
    __shared__ uint32_t s_w[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < n; base += 4096) {
        const int i0 = base + 4 * t;
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < n ? cnt[i0 + k] : 0u;
            sum += v[k];
        }
        uint32_t x = sum;
        x = wave_inclusive_sum(x);
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        uint32_t wbase = 0, total = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t a = s_w[k];
            if (k < w) wbase += a;
            total += a;
        }
        uint32_t run = carry + wbase + (x - sum);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < n) start[i0 + k] = run;
            run += v[k];
        }
        carry += total;
        __syncthreads();
    }
    if (t == 0) start[n] = carry;
}

// Single-block exclusive scan of n values get(i) into put(i, prefix); returns the total.  The
// caller's block has 1024 threads; n up to kScanOneBlock.
template <class G, class P>
__device__ inline uint32_t block_scan_1024(int n, G get, P put, uint32_t* s_w) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < n; base += 4096) {
        const int i0 = base + 4 * t;
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < n ? get(i0 + k) : 0u;
            sum += v[k];
        }
        uint32_t x = sum;
        x = wave_inclusive_sum(x);
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        uint32_t wbase = 0, total = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t a = s_w[k];
            if (k < w) wbase += a;
            total += a;
        }
        uint32_t run = carry + wbase + (x - sum);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < n) put(i0 + k, run);
            run += v[k];
        }
        carry += total;
        __syncthreads();
    }
    return carry;
}

// Work items of the count and emit passes (kNT list entries of a tile each), their exclusive
// scan, and the first capacity check (list entries and items against their buffers), in one
// block: the work of k_tile_items, k_scan1 and k_check_caps stage 1 for up to kScanOneBlock tiles.
__global__ __launch_bounds__(1024) void k_items_scan(const uint32_t* __restrict__ tile_start, int T,
                                                     uint32_t* __restrict__ item_start, Counters* ctr, uint32_t cap_pairs,
                                                     uint32_t cap_items) {
    __shared__ uint32_t s_w[16];
    const uint32_t items = block_scan_1024(
        T, [&](int i) { return (tile_start[i + 1] - tile_start[i] + kNT - 1) / kNT; },
        [&](int i, uint32_t v) { item_start[i] = v; }, s_w);
    if (threadIdx.x == 0) {
        const uint32_t pairs = tile_start[T];
        item_start[T] = items;
        ctr->sizes[0] = pairs;
        ctr->sizes[1] = items;
        if (pairs > cap_pairs || items > cap_items) ctr->cap_overflow = 1u;
    }
}

// The tiles' fragment and batch offsets (exclusive scans of tile_tot and tile_nb) and the
// second capacity check, in one block (k_scan1 twice and k_check_caps stage 2).
__global__ __launch_bounds__(1024) void k_tile_scans(const uint32_t* __restrict__ tile_tot,
                                                     uint32_t* __restrict__ frag_base, const uint32_t* __restrict__ tile_nb,
                                                     uint32_t* __restrict__ batch_start, int T, Counters* ctr,
                                                     uint32_t cap_frags, uint32_t cap_batches) {
    __shared__ uint32_t s_w[16];
    const uint32_t frags = block_scan_1024(
        T, [&](int i) { return tile_tot[i]; }, [&](int i, uint32_t v) { frag_base[i] = v; }, s_w);
    const uint32_t batches = block_scan_1024(
        T, [&](int i) { return tile_nb[i]; }, [&](int i, uint32_t v) { batch_start[i] = v; }, s_w);
    if (threadIdx.x == 0) {
        frag_base[T] = frags;
        batch_start[T] = batches;
        ctr->sizes[2] = frags;
        ctr->sizes[3] = batches;
        if (frags > cap_frags || batches > cap_batches) ctr->cap_overflow = 1u;
    }
}

// The per-pixel counters of a frame: counts 0, key minima ~0, key maxima 0.
// ... and the work-item table of the count and emit passes: item i of tile t (its list chunk
// i - item_start[t]), for the items within the table's capacity.
__global__ void k_fill_pix(uint32_t* __restrict__ cnt, uint32_t* __restrict__ kmin, uint32_t* __restrict__ kmax,
                           uint8_t* __restrict__ thick, size_t n, float4* __restrict__ rgba, size_t n_rgba,
                           const uint32_t* __restrict__ item_start, int T, uint2* __restrict__ item_tab,
                           uint32_t cap_items) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        cnt[i] = 0u;
        kmin[i] = 0xFFFFFFFFu;
        kmax[i] = 0u;
        if (thick) thick[i] = 0;
    }
    // (and the frame's image, transparent black, when one is given)
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rgba; i += (size_t)gridDim.x * blockDim.x)
        rgba[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    // (one wave per tile, its lanes taking the tile's items in turn: a tile can hold thousands
    // of items when a whole groom falls into a few tiles)
    const int lane = threadIdx.x & 63;
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), n_waves = (int)((gridDim.x * blockDim.x) >> 6);
    for (int t = wave; t < T; t += n_waves) {
        const uint32_t i0 = item_start[t], i1 = min(item_start[t + 1], cap_items);
        for (uint32_t i = i0 + lane; i < i1; i += 64) item_tab[i] = make_uint2((uint32_t)t, i - i0);
    }
}

// Multi-block exclusive scan: each 1024-thread block scans kScanChunk counts and leaves its
// total; the totals are scanned by k_scan1; k_scan_add adds each block's base.
__global__ __launch_bounds__(1024) void k_scan_local(const uint32_t* __restrict__ cnt, uint32_t* __restrict__ out,
                                                      uint32_t* __restrict__ part, int n) {
    __shared__ uint32_t s_part[1024];
    const int t = threadIdx.x;
    const int b0 = blockIdx.x * kScanChunk + t * 4;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = b0 + k < n ? cnt[b0 + k] : 0u;
        sum += v[k];
    }
    s_part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t x = t >= off ? s_part[t - off] : 0u;
        __syncthreads();
        s_part[t] += x;
        __syncthreads();
    }
    uint32_t run = s_part[t] - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (b0 + k < n) out[b0 + k] = run;
        run += v[k];
    }
    if (t == 1023) part[blockIdx.x] = s_part[1023];
}

__global__ __launch_bounds__(1024) void k_scan_add(uint32_t* __restrict__ out, const uint32_t* __restrict__ base,
                                                    int n, int nblocks) {
    const int i = blockIdx.x * kScanChunk + threadIdx.x * 4;
    const uint32_t b = base[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i + k < n) out[i + k] += b;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = base[nblocks];
}

// Tile binning without device-wide atomics.  Block b owns the contiguous segment range
// [b per_block, (b + 1) per_block) and counts, in LDS, its segments per tile of the range
// [t0, t0 + nt) (the whole image unless it has more than kMaxLdsTiles tiles); the counts form
// row b of M [nb][T].  A column-wise exclusive scan of M gives each block its place inside
// every tile list, and the scatter pass appends each segment at its block's LDS cursors.
// A tile of the box of a wide segment (radius above 2 px) is kept only if the rectangle of its
// pixel centres meets the segment's footprint (the slab 0 <= t_num <= t_den and the strip
// |cross| <= R sqrt(t_den)): projected on the segment's direction and normal, the four corner
// centres must overlap both.  Exact in integers (corner offsets below 2^15, products below
// 2^30, cross^2 and R^2 t_den in 64 bits); for short, wide segments (thick hairs) this drops
// the many box tiles beyond the segment's ends.  Thin segments keep their box's tiles.
__device__ inline bool tile_meets_footprint(const SegRec& r, int tx, int ty) {
    const int R = (r.hwfx & kHwMask) + 8;
    if (R <= 32) return true;
    const int dx = r.xb - r.xa, dy = r.yb - r.ya;
    const int tden = dx * dx + dy * dy;
    if (tden <= 0) return true;
    const unsigned long long RR = (unsigned long long)(unsigned)(R * R) * (unsigned)tden;
    const int ex0 = 16 * kTile * tx + 8 - r.xa, ex1 = ex0 + 16 * (kTile - 1);
    const int ey0 = 16 * kTile * ty + 8 - r.ya, ey1 = ey0 + 16 * (kTile - 1);
    int tmin = 0x7FFFFFFF, tmax = -0x7FFFFFFF - 1, cmin = 0x7FFFFFFF, cmax = -0x7FFFFFFF - 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int ex = (k & 1) ? ex1 : ex0, ey = (k & 2) ? ey1 : ey0;
        const int tn = ex * dx + ey * dy, cr = ex * dy - ey * dx;
        tmin = min(tmin, tn);
        tmax = max(tmax, tn);
        cmin = min(cmin, cr);
        cmax = max(cmax, cr);
    }
    if (tmax < 0 || tmin > tden) return false;
    if (cmin > 0 && (unsigned long long)((long long)cmin * cmin) >= RR) return false;
    if (cmax < 0 && (unsigned long long)((long long)cmax * cmax) >= RR) return false;
    return true;
}

template <class F>
__device__ inline void for_each_tile_in_range(const SegRec& r, int ntx, int nty, int t0, int nt, F&& f) {
    if (!(r.hwfx & kFlagVisible)) return;
    const TileRect rc = tile_rect(r, ntx, nty);
    for (int ty = rc.ty0; ty <= rc.ty1; ++ty)
        for (int tx = rc.tx0; tx <= rc.tx1; ++tx) {
            const int l = ty * ntx + tx - t0;
            if ((unsigned)l < (unsigned)nt && tile_meets_footprint(r, tx, ty)) f(l);
        }
}

// The first pass also leaves per-block segment statistics in blk[b] = (visible, culled as too
// long, bits of the largest visible half-width) for k_bin_offsets to reduce.
__global__ __launch_bounds__(kBinThreads) void k_bin_count(const SegRec* __restrict__ seg, int nseg, int per_block,
                                                           int ntx, int nty, int t0, int nt,
                                                           uint32_t* __restrict__ M, uint4* __restrict__ blk) {
    extern __shared__ uint32_t s_tc[];
    __shared__ uint32_t s_maxhw;
    const int T = ntx * nty;
    for (int i = threadIdx.x; i < nt; i += kBinThreads) s_tc[i] = 0;
    if (threadIdx.x == 0) s_maxhw = 0;
    __syncthreads();
    const int g0 = blockIdx.x * per_block, g1 = min(nseg, g0 + per_block);
    uint32_t nvis = 0, nlong = 0, nsplit = 0, maxhw = 0;
    for (int g = g0 + (int)threadIdx.x; g < g1; g += kBinThreads) {
        const SegRec r = seg[g];
        if (r.hwfx & kFlagVisible) {
            ++nvis;
            maxhw = max(maxhw, __float_as_uint(r.hw));
        }
        nlong += (r.hwfx & kFlagCulledLong) ? 1u : 0u;
        nsplit += (r.hwfx & kFlagSplit) ? 1u : 0u;
        for_each_tile_in_range(r, ntx, nty, t0, nt, [&](int l) { atomicAdd(&s_tc[l], 1u); });
    }
    if (t0 == 0) {
        if (maxhw) atomicMax(&s_maxhw, maxhw);
        uint32_t v = nvis, c = nlong, sp = nsplit;
        for (int off = 32; off >= 1; off >>= 1) {
            v += __shfl_xor(v, off);
            c += __shfl_xor(c, off);
            sp += __shfl_xor(sp, off);
        }
        __shared__ uint32_t s_v[kBinThreads / 64], s_c[kBinThreads / 64], s_sp[kBinThreads / 64];
        if ((threadIdx.x & 63) == 0) {
            s_v[threadIdx.x >> 6] = v;
            s_c[threadIdx.x >> 6] = c;
            s_sp[threadIdx.x >> 6] = sp;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tv = 0, tc = 0, ts = 0;
            for (int w = 0; w < kBinThreads / 64; ++w) {
                tv += s_v[w];
                tc += s_c[w];
                ts += s_sp[w];
            }
            blk[blockIdx.x] = make_uint4(tv, tc, s_maxhw, ts);
        }
    }
    __syncthreads();
    uint32_t* row = M + (size_t)blockIdx.x * T + t0;
    for (int i = threadIdx.x; i < nt; i += kBinThreads) row[i] = s_tc[i];
}

// Column-wise exclusive scan of M: M[b][t] <- sum of M[b'][t] over b' < b, tot[t] = column sum.
// A block takes 64 tiles (one per lane) and its 16 waves split the rows into 16 ranges: each
// wave sums its range, the range offsets come from LDS, and a second walk writes the prefixes.
// Block 0 also reduces the per-block segment statistics into ctr.
__global__ __launch_bounds__(1024) void k_bin_offsets(uint32_t* __restrict__ M, int nb, int T,
                                                      uint32_t* __restrict__ tot, const uint4* __restrict__ blk,
                                                      Counters* __restrict__ ctr) {
    __shared__ uint32_t s_part[16][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + lane;
    const int rows = (nb + 15) / 16, r0 = min(nb, w * rows), r1 = min(nb, r0 + rows);
    uint32_t sum = 0;
    if (t < T) {
#pragma unroll 8
        for (int b = r0; b < r1; ++b) sum += M[(size_t)b * T + t];
    }
    s_part[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, total = 0;
    for (int w2 = 0; w2 < 16; ++w2) {
        const uint32_t v = s_part[w2][lane];
        if (w2 < w) run += v;
        total += v;
    }
    if (t < T) {
        for (int b = r0; b < r1; ++b) {
            const size_t q = (size_t)b * T + t;
            const uint32_t v = M[q];
            M[q] = run;
            run += v;
        }
        if (w == 0) tot[t] = total;
    }
    if (blockIdx.x == 0 && w == 0) {
        uint32_t v = 0, c = 0, m = 0, sp = 0;
        for (int b = lane; b < nb; b += 64) {
            const uint4 x = blk[b];
            v += x.x;
            c += x.y;
            m = max(m, x.z);
            sp += x.w;
        }
        for (int off = 32; off >= 1; off >>= 1) {
            v += __shfl_xor(v, off);
            c += __shfl_xor(c, off);
            m = max(m, (uint32_t)__shfl_xor((int)m, off));
            sp += __shfl_xor(sp, off);
        }
        if (lane == 0) {
            ctr->visible = v;
            ctr->culled_long = c;
            ctr->max_hw_bits = m;
            ctr->split_needed = sp;
        }
    }
}

__global__ __launch_bounds__(kBinThreads) void k_scatter(const SegRec* __restrict__ seg, int nseg, int per_block,
                                                         int ntx, int nty, int t0, int nt,
                                                         const uint32_t* __restrict__ tile_start,
                                                         const uint32_t* __restrict__ M, uint32_t* __restrict__ list,
                                                         const Counters* __restrict__ ctr) {
    extern __shared__ uint32_t s_tc[];
    if (ctr->cap_overflow) return;
    const int T = ntx * nty;
    const uint32_t* row = M + (size_t)blockIdx.x * T + t0;
    for (int i = threadIdx.x; i < nt; i += kBinThreads) s_tc[i] = tile_start[t0 + i] + row[i];
    __syncthreads();
    const int g0 = blockIdx.x * per_block, g1 = min(nseg, g0 + per_block);
    for (int g = g0 + (int)threadIdx.x; g < g1; g += kBinThreads)
        for_each_tile_in_range(seg[g], ntx, nty, t0, nt, [&](int l) { list[atomicAdd(&s_tc[l], 1u)] = (uint32_t)g; });
}

// The frame's sizes against the buffers' capacities (one thread).
__global__ void k_check_caps(FrameBufs f, FrameCaps caps, int stage) {
    if (threadIdx.x != 0) return;
    uint32_t over = 0;
    if (stage == 1) {
        const uint32_t pairs = f.tile_start[f.T], items = f.item_start[f.T];
        f.ctr->sizes[0] = pairs;
        f.ctr->sizes[1] = items;
        over = (pairs > caps.pairs) || (items > caps.items);
    } else {
        const uint32_t frags = f.frag_base[f.T], batches = f.batch_start[f.T];
        f.ctr->sizes[2] = frags;
        f.ctr->sizes[3] = batches;
        over = (frags > caps.frags) || (batches > caps.batches);
    }
    if (over) f.ctr->cap_overflow = 1u;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------------------
// Coverage: every fragment of a tile's segments, with the work shared across a wave.  A
// segment's pixels are taken one line at a time along its major axis (rows when |dy| >= |dx|,
// else columns; u names the major axis, v the minor one), and the lanes of a wave share out all
// its (segment, line) pairs, 64 per round, so that a wave does not run as long as its longest
// segment.  On a line the covered pixels are exactly those of the segment's box (widened by the
// radius, clipped to the tile and the image) whose centre passes the integer predicate
// 0 <= t_num < t_den and cross^2 < R^2 t_den.  Along a line both t_num and cross are linear in
// the minor index (steps 16 dv and 16 du per pixel; t_num and |cross| are symmetric under the
// exchange of x and y, so one predicate serves both orientations), so each condition holds on
// an interval of the minor index, and the line's fragments are the intersection of three
// intervals: no candidate is tested one by one.
//
// 32-bit integers are exact here: endpoints lie inside the guard band, |dx|, |dy| <= kMaxAxis
// (longer segments are drawn as pieces), the radius is <= kMaxHwFx + 8 and every pixel centre
// of the widened box lies within kMaxAxis + kMaxHwFx + 24 < 2^16 sub-pixels of the first
// endpoint on each axis, so each product e dv, e du is below 2^30 and t_num, cross are below
// 2^31 (the products take the 24-bit multiplier: operands below 2^23); s_max < 2^30 and
// t_den < 2^30.  cross^2 < R^2 t_den is decided as |cross| <= s_max =
// floor(sqrt(R^2 t_den - 1)), found per segment in 64-bit integers.  x >> 4 is floor(x / 16).
//
// The interval ends are floor divisions n / d with d = 16 |du| or 16 |dv| (<= 2^18), exact:
// only quotients in [-17, 17] matter (a line has at most 16 pixels in a tile), and there n is
// below 2^23 in magnitude, so float(n) is exact; q = floor(n / d - 2^-16) from the hardware
// reciprocal is then floor(n / d) or one less (the reciprocal and the fused multiply-add err by
// under 3e-6 on quotients of that size, less than the 2^-16 bias), and one exact integer test,
// (q + 1) d <= n, settles it.  Quotients beyond [-17, 17] are clamped to +-17 before the test
// and stay on their side.
struct CovSetup {
    int4 g0;     // (c0, t0, dc, dt): cross and t_num at the box's first minor pixel of line l = 0
                 // and their steps per line, each sign-normalised (c by the sign of du, t by
                 // that of dv) so that both grow with the minor index at 16 |du| and 16 |dv|
    int4 g1;     // (s_max, lo, hi, first line - lines before this lane in the wave): the slab
                 // lo <= t <= hi is 0 <= t_num <= t_den - 1 after the sign normalisation
    float4 g2;   // (1 / (16 |du|), 1 / max(16 |dv|, 1), bits of 16 |du|,
                 //  bits of 16 |dv| | first pixel (8 bits) << 19 | last minor offset (4 bits) << 27 | steep << 31)
};

// The largest s with s^2 < R^2 t_den (R^2 t_den >= 64): a square root, corrected in 64-bit
// integers, so that |cross| <= s_max is exactly cross^2 < R^2 t_den.  Below 2^48 (every
// strand) the float square root is within 3 of s (relative error under 2^-22 on s < 2^24),
// above it the double one.
__device__ inline int strip_smax(int R, int tden) {
    const unsigned long long lim = (unsigned long long)(unsigned)(R * R) * (unsigned)tden - 1ull;
    unsigned long long s = lim < (1ull << 48) ? (unsigned long long)__builtin_amdgcn_sqrtf((float)lim)
                                              : (unsigned long long)sqrt((double)lim);
    while (s * s > lim) --s;
    while ((s + 1) * (s + 1) <= lim) ++s;
    return (int)min(s, 0x7FFFFFFFull);
}
constexpr int kCovLinesPerWave = 64 * kTile;   // a segment has at most kTile lines in a tile

// floor(n / d) for 1 <= d <= 2^18 where it lies in [-17, 17]; a quotient beyond that range
// comes back beyond [-17, 16] on its own side.  rd: the hardware reciprocal of d.
__device__ inline int floordiv_small(int n, int d, float rd) {
    float qf = floorf(fmaf((float)n, rd, -0x1p-16f));
    qf = fminf(fmaxf(qf, -17.0f), 17.0f);
    const int q = (int)qf;
    return q + ((__mul24(q, d) + d <= n) ? 1 : 0);
}

// Stages lane t's segment (valid: the lane holds one) in s_cov[t], numbers the wave's lines
// and records each line's lane in s_own (kCovLinesPerWave bytes per wave); returns the wave's
// line count.  Ends with a block barrier (all threads must call it).
__device__ inline uint32_t cov_setup(const SegRec& s, bool valid, int px0, int py0, int W, int H, CovSetup* s_cov,
                                     uint8_t* s_own) {
    const int t = threadIdx.x, lane = t & 63;
    uint32_t nl = 0;
    CovSetup c{};
    if (valid) {
        const int dx = s.xb - s.xa, dy = s.yb - s.ya;
        const int tden = dx * dx + dy * dy;
        const int R = (s.hwfx & kHwMask) + 8;
        const int i0 = max(px0, ((min(s.xa, s.xb) - R - 8) >> 4) + 1);
        const int i1 = min(min(px0 + kTile, W) - 1, ((max(s.xa, s.xb) + R - 8 + 15) >> 4) - 1);
        const int j0 = max(py0, ((min(s.ya, s.yb) - R - 8) >> 4) + 1);
        const int j1 = min(min(py0 + kTile, H) - 1, ((max(s.ya, s.yb) + R - 8 + 15) >> 4) - 1);
        if (tden > 0 && i0 <= i1 && j0 <= j1) {
            const bool steep = abs(dy) >= abs(dx);
            const int au = steep ? s.ya : s.xa, av = steep ? s.xa : s.ya;
            const int du = steep ? dy : dx, dv = steep ? dx : dy;
            nl = (uint32_t)(steep ? j1 - j0 + 1 : i1 - i0 + 1);
            const int vmin = steep ? i0 : j0, vmax = steep ? i1 : j1;
            const int u0 = steep ? j0 : i0;
            const int eu = 16 * u0 + 8 - au, ev = 16 * vmin + 8 - av;
            const int tn = __mul24(ev, dv) + __mul24(eu, du);   // t_num at (u0, vmin)
            const int cr = __mul24(ev, du) - __mul24(eu, dv);   // cross at (u0, vmin)
            // per line eu grows by 16: t_num by 16 du, cross by -16 dv
            const int sgu = du < 0 ? -1 : 1, sgv = dv < 0 ? -1 : 1;
            const int B = 16 * abs(du), A = 16 * abs(dv);
            const int lu = u0 - (steep ? py0 : px0), lv = vmin - (steep ? px0 : py0);   // 0..15
            const int pix0 = steep ? lu * kTile + lv : lv * kTile + lu;
            c.g0 = make_int4(sgu * cr, sgv * tn, -16 * sgu * dv, 16 * sgv * du);
            c.g1 = make_int4(strip_smax(R, tden), dv < 0 ? 1 - tden : 0, dv < 0 ? 0 : tden - 1, 0);
            c.g2 = make_float4(__builtin_amdgcn_rcpf((float)B), __builtin_amdgcn_rcpf((float)max(A, 1)),
                               __int_as_float(B),
                               __int_as_float(A | pix0 << 19 | (vmax - vmin) << 27 | (steep ? (int)0x80000000u : 0)));
        }
    }
    uint32_t x = nl;
    x = wave_inclusive_sum(x);
    const uint32_t excl = x - nl;
    c.g1.w = -(int)excl;     // line index = g1.w + the wave-wide line number
    s_cov[t] = c;
    uint8_t* own = s_own + (t >> 6) * kCovLinesPerWave;
    for (uint32_t r = 0; r < nl; ++r) own[excl + r] = (uint8_t)lane;
    const uint32_t total = __shfl(x, 63);
    __syncthreads();
    return total;
}

// Calls f(p, tnum, tden, owner) for every fragment of the wave's segments in this tile (p: the
// pixel's index in the tile; owner: the block thread whose segment it is).  total and the
// staging from cov_setup.
template <class F>
__device__ inline void wave_coverage(const CovSetup* s_cov, const uint8_t* s_own, uint32_t total, F&& f) {
    const int t = threadIdx.x, lane = t & 63, wbase = t & ~63;
    const uint8_t* own = s_own + (t >> 6) * kCovLinesPerWave;
    for (uint32_t g = (uint32_t)lane; g < total; g += 64) {
        const int o = wbase + own[g];
        const CovSetup c = s_cov[o];
        const int l = c.g1.w + (int)g;                       // line within the box, 0..15
        const int cl = c.g0.x + __mul24(l, c.g0.z);          // at the box's first minor pixel
        const int tl = c.g0.y + __mul24(l, c.g0.w);
        const int smax = c.g1.x, lo = c.g1.y, hi = c.g1.z;
        const int B = __float_as_int(c.g2.z);
        const int bits = __float_as_int(c.g2.w);
        const int A = bits & 0x7FFFF;
        // strip: -s_max <= cl + x B <= s_max; slab: lo <= tl + x A <= hi.  Values that leave
        // a condition false on all of x = 0..15 are clamped to just beyond that range first, so
        // that the numerators stay below 2^31.
        const int m = smax + 16 * B;
        const int cc = min(max(cl, -m), m);
        int x0 = max(0, -floordiv_small(smax + cc, B, c.g2.x));
        int x1 = min((bits >> 27) & 15, floordiv_small(smax - cc, B, c.g2.x));
        if (A > 0) {
            const int tc = min(max(tl, lo - 16 * A), hi + 1);
            x0 = max(x0, -floordiv_small(tc - lo, A, c.g2.y));
            x1 = min(x1, floordiv_small(hi - tc, A, c.g2.y));
        } else if (tl < lo || tl > hi) {
            x1 = -1;
        }
        if (x0 > x1) continue;
        const int tden = hi - lo + 1;
        const int sv = bits < 0 ? 1 : kTile;                  // pixel step along the minor axis
        int p = ((bits >> 19) & 0xFF) + __mul24(l, bits < 0 ? kTile : 1) + __mul24(x0, sv);
        // t_num itself: the normalised t times the sign of dv (lo < 0 exactly when dv < 0, as
        // then t_den >= 2)
        const int sgn = lo < 0 ? -1 : 1;
        int tnum = sgn * (tl + __mul24(x0, A));
        const int tstep = sgn * A;
        for (int xx = x0; xx <= x1; ++xx, p += sv, tnum += tstep) f(p, tnum, tden, o);
    }
}

__device__ inline uint32_t depth_key_iz(float iza, float izb, int tnum, int tden) {
    const float t = (float)tnum / (float)tden;
    const float iz = iza + t * (izb - iza);
    return 0xFFFFFFFFu - __float_as_uint(iz);
}

// The global segment id of a fragment record's second word (see FrameBufs::gid): the record
// holds it, or the index of the segment in the tile's list.
__device__ inline uint32_t seg_of(uint32_t y, const uint32_t* list, bool gid) {
    return gid ? (y & 0xFFFFFFu) : list[y & 0xFFFFFFu];
}

struct ShadeArgs {
    CamConst cam;
    LightsConst lights;
    MatConst mat;
    const SegRec* seg;
    const ShadeRec* shade;
};

// Deep opacity map lookup (the shadow pass's count of hairs in front of a point toward a
// light).  Both helpers round every operation once, in this order, so the lookup position and
// its texel weights are the ones the integer raster parameter fixes (fragment's point on the
// centre line: t from the integer parameter, perspective-correct t_w, x = pA + t_w (pB - pA)).
__device__ inline void dom_point(const SegRec& s, const float4& q0, const float4& q1, int tnum, int tden, float& x,
                                 float& y, float& z) {
    const float t = (float)tnum / (float)tden;
    const float iz = s.iza + t * (s.izb - s.iza);
    const float tw = (t * s.izb) / iz;
    x = q0.x + tw * (q1.x - q0.x);
    y = q0.y + tw * (q1.y - q0.y);
    z = q0.z + tw * (q1.z - q0.z);
}

// Entry i of (0, A.y, A.z, A.w, B.x, B.y, B.z, B.w) = (C_{-1}, C_0 .. C_6) of a texel.
__device__ inline float texel_c(const float4& A, const float4& B, int i) {
    float v = 0.0f;
    v = i == 1 ? A.y : v;
    v = i == 2 ? A.z : v;
    v = i == 3 ? A.w : v;
    v = i == 4 ? B.x : v;
    v = i == 5 ? B.y : v;
    v = i == 6 ? B.z : v;
    v = i == 7 ? B.w : v;
    return v;
}

// delta = |cross| / (16 sqrt(t_den)), the pixel centre's distance from the centre line in pixels,
// in double: the hardware reciprocal square root refined by one Newton step (relative error
// near 2^-46).
__device__ inline double delta_d(int cr, int tden) {
    const double x = (double)tden;
    double r = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x * r;
    r = fma(r, fma(-hx, r, 0.5), r);
    return fabs((double)cr) * r * 0.0625;
}

// A strand's coverage alpha = min(hw + delta, 1/2) - max(delta - hw, -1/2), clamped to [0, 1]:
// at an edge pixel of low coverage it is a small difference of numbers near 1/2, so it is
// evaluated in double and rounded to float once, and its relative error stays at float
// precision however small the coverage.
__device__ inline float strand_alpha(int cr, int tden, float hw, float& delta) {
    const double dd = delta_d(cr, tden);
    delta = (float)dd;
    const double h = (double)hw;
    return (float)fmin(fmax(fmin(h + dd, 0.5) - fmax(dd - h, -0.5), 0.0), 1.0);
}

// Hairs in front of (x, y, z): per texel, x_l = (iz0 - iz) / delta - 1 layers behind the first
// hit (one layer of bias), C_{j-1} + (x_l - j)(C_j - C_{j-1}) inside layer j, C_{K-1} beyond;
// bilinear over the four nearest texel centres; outside the grid or on empty texels 0.
__device__ inline float dom_count(const DomView& dv, float x, float y, float z) {
    const DomGrid& g = *dv.grid;
    const float u = dot_e(g.b.e1, x, y, z), v = dot_e(g.b.e2, x, y, z);
    const float izp = g.z_ref - dot_e(g.b.d, x, y, z);
    const float Tx = (u - g.u0) / g.s - 0.5f, Ty = (v - g.v0) / g.s - 0.5f;
    const float i0f = floorf(Tx), j0f = floorf(Ty);
    const float fx = Tx - i0f, fy = Ty - j0f;
    const int i0 = (int)i0f, j0 = (int)j0f;
    float n = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int i = i0 + (c & 1), j = j0 + (c >> 1);
        if (i < 0 || j < 0 || i >= g.R || j >= g.R) continue;
        const size_t o = 2 * ((size_t)j * g.R + i);
        const float4 A = dv.tex[o];
        if (!(A.x > 0.0f)) continue;
        const float xl = (A.x - izp) / dv.delta - 1.0f;
        if (!(xl >= 0.0f)) continue;
        const float4 B = dv.tex[o + 1];
        float val;
        if (xl >= (float)dv.K) {
            val = texel_c(A, B, dv.K);
        } else {
            const int jl = (int)floorf(xl);
            const float Cp = texel_c(A, B, jl), Cj = texel_c(A, B, jl + 1);
            val = Cp + (xl - (float)jl) * (Cj - Cp);
        }
        const float w = ((c & 1) ? fx : 1.0f - fx) * ((c >> 1) ? fy : 1.0f - fy);
        n += w * val;
    }
    return n;
}

// Radiance (RGB), coverage alpha and cross-section offset h of one fragment, written once over
// the scalar type T: float for rendering, Dual<N> for the backward pass.  T carries the
// fitted parameters (half-width hw, semi-axes |a|, |b|, hair radius r, absorption); the view
// geometry (frame, angles) does not depend on them and stays float.
template <int KIND, int MODEL, class T, bool SHADOW = false>
__device__ inline void shade_core(const ShadeArgs& a, const SegRec& s, const float4& q0, const float4& q1,
                                  const float4& q2, float n_total, int pxg, int pyg, const T& hw, const T& a_len,
                                  const T& b_len, const T& rr, const T sig[3], T& alpha, T& hoff, T L[3]) {
#pragma clang fp contract(fast)
    // integer coverage geometry; 32 bits suffice because a covered pixel centre lies within
    // the segment's box widened by its radius and longer segments (kMaxAxis) are culled
    const int ex = 16 * pxg + 8 - s.xa, ey = 16 * pyg + 8 - s.ya;
    const int dx = s.xb - s.xa, dy = s.yb - s.ya;
    const int tnum = ex * dx + ey * dy, tden = dx * dx + dy * dy;
    const int cr = ex * dy - ey * dx;
    // (the coverage decision was taken exactly when the fragment was emitted; what follows is
    // continuous, so it uses the hardware reciprocal and reciprocal square root)
    float delta;
    if constexpr (KIND == 1) {
        // a thick hair is many pixels wide, so at its footprint's edge alpha = 1/2 - (delta - hw)
        // is a small difference of large numbers; delta is carried as a float pair (hi + lo) from
        // a double evaluation, and hi - hw is exact there (Sterbenz), which keeps alpha's
        // absolute error at the level of a strand's instead of an ulp of the hair width
        const double dd = delta_d(cr, tden);
        delta = (float)dd;
        const float dlo = (float)(dd - (double)delta);
        const T d_minus = (delta - hw) + dlo, d_plus = (hw + delta) + dlo;
        alpha = m_min(m_max(m_min(d_plus, T(0.5f)) - m_max(d_minus, T(-0.5f)), T(0.0f)), T(1.0f));
    } else {
        alpha = strand_alpha(cr, tden, hw, delta);
    }
    float sgn = cr > 0 ? 1.0f : (cr < 0 ? -1.0f : 0.0f);
    if (s.hwfx & kFlagNegSide) sgn = -sgn;
    const T h = m_min(m_max((sgn * delta) * m_rcp(hw + 0.5f), T(-1.0f)), T(1.0f));
    hoff = h;
    // the world parameter of the fragment's screen parameter t = t_num / t_den: inverse depth is
    // affine on screen, so t_w = t izB / (izA + t (izB - izA)), here with t_den cleared
    const float ftn = (float)tnum;
    const float tw = ftn * s.izb * m_rcp((float)tden * s.iza + ftn * (s.izb - s.iza));

    // fibre frame at the fragment's world point
    const V3<float> pA = v3(q0.x, q0.y, q0.z);
    const V3<float> d = sub(v3(q1.x, q1.y, q1.z), pA);
    const V3<float> u = scale(d, m_rsqrt(dot(d, d)));
    const V3<float> xw = v3(pA.x + tw * d.x, pA.y + tw * d.y, pA.z + tw * d.z);
    V3<float> wo = sub(v3(a.cam.pos[0], a.cam.pos[1], a.cam.pos[2]), xw);
    wo = scale(wo, m_rsqrt(dot(wo, wo)));
    const float dwu = dot(wo, u);
    V3<float> wp = sub(wo, scale(u, dwu));
    float wpn2 = dot(wp, wp);
    // the longitudinal angle from both of its legs: atan2(sin, |w_perp|) stays accurate where
    // asin(sin) loses digits (views and lights close to the fibre axis, where the narrow
    // longitudinal lobes are most sensitive to theta)
    float r_wp = m_rsqrt(wpn2);
    const float cos_to = wpn2 > 0.0f ? wpn2 * r_wp : 0.0f;   // |w_perp|
    const bool degen = wpn2 < 1e-14f;
    if (degen) {  // view along the fibre: any normal direction; phi is set to 0
        const float ax = fabsf(u.x), ay = fabsf(u.y), az = fabsf(u.z);
        V3<float> e = (ax <= ay && ax <= az) ? v3(1.f, 0.f, 0.f) : (ay <= az ? v3(0.f, 1.f, 0.f) : v3(0.f, 0.f, 1.f));
        wp = sub(e, scale(u, dot(e, u)));
        wpn2 = dot(wp, wp);
        r_wp = m_rsqrt(wpn2);
    }
    const V3<float> xh = scale(wp, r_wp);
    const V3<float> yh = cross(u, xh);
    const float sin_to = fminf(fmaxf(dwu, -1.0f), 1.0f);
    const T gamma_o = m_asin(h);
    const T cgo = m_sqrt((1.0f - h) * (1.0f + h));
    const T sigl[3] = {sig[0] * kLog2e, sig[1] * kLog2e, sig[2] * kLog2e};

    ClusterFrag<T> cf;
    T W, ia, ib;
    V3<float> ah{}, bh{};
    if (KIND == 1) {
        ah = v3(q2.x, q2.y, q2.z);
        bh = cross(u, ah);
        const T pa = a_len * dot(ah, yh), pb = b_len * dot(bh, yh);
        W = m_sqrt(pa * pa + pb * pb);
        ia = m_rcp(a_len);
        ib = m_rcp(b_len);
        cf.n_total = T(n_total);
        cf.rho = m_min(m_max(n_total * rr * rr * (ia * ib), T(0.0f)), T(1.0f));
    }
    float dpx = 0.f, dpy = 0.f, dpz = 0.f;
    if (SHADOW) dom_point(s, q0, q1, tnum, tden, dpx, dpy, dpz);
    L[0] = L[1] = L[2] = T(0.0f);
    for (int li = 0; li < a.lights.n; ++li) {
        const LightConst& lc = a.lights.l[li];
        V3<float> wi;
        float E[3];
        if (lc.kind == 0) {
            wi = v3(lc.vec[0], lc.vec[1], lc.vec[2]);
            E[0] = lc.rgb[0]; E[1] = lc.rgb[1]; E[2] = lc.rgb[2];
        } else {
            const V3<float> dl = sub(v3(lc.vec[0], lc.vec[1], lc.vec[2]), xw);
            const float inv = m_rsqrt(dot(dl, dl));
            wi = scale(dl, inv);
            const float i2 = inv * inv;
            E[0] = lc.rgb[0] * i2; E[1] = lc.rgb[1] * i2; E[2] = lc.rgb[2] * i2;
        }
        const float sin_ti = dot(wi, u);
        const LightView v = light_view(sin_ti, sin_to, cos_to, dot(wi, xh), dot(wi, yh), degen, a.mat);
        // hairs between the light and this fragment (shadow pass), added to the forward count
        const float ns = (SHADOW && a.lights.dom[li].grid) ? dom_count(a.lights.dom[li], dpx, dpy, dpz) : 0.0f;
        T f[3];
        if (KIND == 0 && SHADOW && ns > 0.0f) {
            ClusterFrag<T> c1;
            c1.n_total = T(1.0f);
            c1.rho = T(1.0f);
            c1.n_F = T(1.0f + ns);
            c1.n_B = T(1.0f);
            if (MODEL == 0)
                f_ours(v, h, gamma_o, cgo, sigl, a.mat, c1, f);
            else
                f_ours_rttd(v, a.mat, c1, f);
        } else if (KIND == 0) {
            if (MODEL == 0)
                f_single(v, h, gamma_o, cgo, sigl, a.mat, f);
            else
                f_single_rttd(v, a.mat, f);
        } else {
            // chord of the view ray's entry point toward the light, in the cross-section
            const V3<float> Dp = sub(wi, scale(u, sin_ti));
            const float dn2 = dot(Dp, Dp);
            T s_star(0.0f);
            if (dn2 > 1e-14f) {
                const V3<float> D = scale(Dp, m_rsqrt(dn2));
                const T oa = h * W * dot(yh, ah) * ia, ob = h * W * dot(yh, bh) * ib;
                const T xa = dot(xh, ah) * ia, xb = dot(xh, bh) * ib;
                const T qa = xa * xa + xb * xb, qb = oa * xa + ob * xb, qc = oa * oa + ob * ob - 1.0f;
                const T disc = m_max(qb * qb - qa * qc, T(0.0f));
                const T tt = (qb - m_sqrt(disc)) * m_rcp(qa);
                const T Pa = oa - tt * xa, Pb = ob - tt * xb;
                const T Da = dot(D, ah) * ia, Db = dot(D, bh) * ib;
                s_star = -2.0f * (Pa * Da + Pb * Db) * m_rcp(Da * Da + Db * Db);
            }
            const T kappa = m_sqrt(n_total * (1.0f / kPi) * (ia * ib));
            const T lF = m_max(s_star, T(0.0f)), lB = m_max(-s_star, T(0.0f));
            const bool back = fabsf(v.phi) < 0.5f * kPi;
            cf.n_F = (back || n_total < 2.0f) ? T(1.0f) : m_max(cf.rho * kappa * lF, T(1.0f));
            cf.n_B = m_max(cf.rho * kappa * lB, T(1.0f));
            if (SHADOW) cf.n_F = cf.n_F + ns;
            if (MODEL == 0)
                f_ours(v, h, gamma_o, cgo, sigl, a.mat, cf, f);
            else
                f_ours_rttd(v, a.mat, cf, f);
        }
        L[0] = L[0] + (E[0] * v.cos_ti) * f[0];
        L[1] = L[1] + (E[1] * v.cos_ti) * f[1];
        L[2] = L[2] + (E[2] * v.cos_ti) * f[2];
    }
}

// KIND 0: strands, 1: thick hairs, 2: a mixed frame (the segment's flag decides).
// MODEL 0: near-field R / TT / TRT, 1: R / TT / D.
// A fragment's segment inputs (integer record and shading record), fetched ahead of use.
struct SegInputs {
    SegRec s;
    float4 q0, q1, q2, q3;
};

// KIND 0 (a strand-level frame) reads the packed strand record alone; the others read the
// screen record and the ShadeRec.
template <int KIND>
__device__ inline SegInputs fetch_segment(const ShadeArgs& a, uint32_t gseg) {
    SegInputs r;
    const ShadeRec& sr = a.shade[gseg];
    if (KIND == 0) {
        const float4 p0 = sr.q0, p1 = sr.q1, p2 = sr.q2, p3 = sr.q3;
        r.s.xa = __float_as_int(p0.x);
        r.s.ya = __float_as_int(p0.y);
        r.s.xb = __float_as_int(p0.z);
        r.s.yb = __float_as_int(p0.w);
        r.s.iza = p1.x;
        r.s.izb = p1.y;
        r.s.hw = fabsf(p1.z);
        r.s.hwfx = (__float_as_uint(p1.z) >> 31) ? kFlagNegSide : 0;
        r.q0 = make_float4(p1.w, p2.x, p2.y, p3.y);
        r.q1 = make_float4(p2.z, p2.w, p3.x, p3.z);
        r.q2 = make_float4(0.f, 0.f, 0.f, p3.w);
        r.q3 = make_float4(0.f, 0.f, 0.f, 0.f);
        return r;
    }
    r.s = a.seg[gseg];
    r.q0 = sr.q0;
    r.q1 = sr.q1;
    r.q2 = sr.q2;
    r.q3 = sr.q3;
    return r;
}

template <int KIND, int MODEL, bool SHADOW = false>
__device__ inline void shade_inputs(const ShadeArgs& a, const SegInputs& in, int pxg, int pyg, float& alpha,
                                    float& hoff, float L[3]) {
    const float sig[3] = {in.q0.w, in.q1.w, in.q2.w};
    if (KIND == 0 || KIND == 3 || (KIND == 2 && !(in.s.hwfx & kFlagThick))) {
        shade_core<0, MODEL, float, SHADOW>(a, in.s, in.q0, in.q1, in.q2, 1.0f, pxg, pyg, in.s.hw, 0.f, 0.f, 0.f, sig, alpha,
                                    hoff, L);
    } else {
        shade_core<1, MODEL, float, SHADOW>(a, in.s, in.q0, in.q1, in.q2, in.q3.z, pxg, pyg, in.s.hw, in.q3.x, in.q3.y, in.q3.w,
                                    sig, alpha, hoff, L);
    }
}

template <int KIND, int MODEL>
__device__ inline void shade_fragment(const ShadeArgs& a, uint32_t gseg, int pxg, int pyg, float& alpha, float& hoff,
                                      float L[3]) {
    shade_inputs<KIND, MODEL>(a, fetch_segment<KIND>(a, gseg), pxg, pyg, alpha, hoff, L);
}

// Block-wide exclusive scan of one uint per thread (256 threads); returns the total.
__device__ inline uint32_t block_exscan_u32(uint32_t v, uint32_t* s_tmp, uint32_t& excl) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t x = v;
    x = wave_inclusive_sum(x);
    if (lane == 63) s_tmp[wv] = x;
    __syncthreads();
    uint32_t base = 0, total = 0;
#pragma unroll
    for (int w2 = 0; w2 < kNT / 64; ++w2) {
        const uint32_t a = s_tmp[w2];
        if (w2 < wv) base += a;
        total += a;
    }
    __syncthreads();
    excl = base + x - v;
    return total;
}

#ifdef HAIR_PHASE_STATS
#define PHASE_BEGIN() unsigned long long ph_t0 = wall_clock64()
// (the barrier here only makes the timing cover the whole block; correctness never relies on it)
#define PHASE_END(ctr, i)                                                      \
    do {                                                                       \
        __syncthreads();                                                       \
        if (threadIdx.x == 0) atomicAdd(&(ctr)->phase[i], wall_clock64() - ph_t0); \
        ph_t0 = wall_clock64();                                                \
    } while (0)
#define PHASE_RESET() ph_t0 = wall_clock64()
#define PHASE_ADD(ctr, i, v) do { if (threadIdx.x == 0) atomicAdd(&(ctr)->phase[i], (unsigned long long)(v)); } while (0)
#else
#define PHASE_BEGIN() do {} while (0)
#define PHASE_END(ctr, i) do {} while (0)
#define PHASE_RESET() do {} while (0)
#define PHASE_ADD(ctr, i, v) do {} while (0)
#endif

// Work items of the count and emit kernels: chunks of kNT consecutive entries of a tile list.
__global__ __launch_bounds__(256) void k_tile_items(const uint32_t* __restrict__ tile_start, int T,
                                                    uint32_t* __restrict__ items) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const uint32_t n = tile_start[t + 1] - tile_start[t];
    items[t] = (n + kNT - 1) / kNT;
}

// Count pass: per-pixel fragment counts of each tile.  Each item adds its LDS-aggregated
// counts to the tile's pixels and keeps the returned base (its slice of every pixel's range).
__global__ __launch_bounds__(kNT) void k_count(FrameBufs f, CamConst cam) {
    __shared__ uint32_t s_cnt[kTilePix];
    __shared__ CovSetup s_cov[kNT];
    __shared__ uint8_t s_own[kNT / 64 * kCovLinesPerWave];
    PHASE_BEGIN();
    const uint32_t n_items = f.item_start[f.T];
    if (blockIdx.x >= n_items || f.ctr->cap_overflow) return;
    const uint32_t item = xcd_contiguous(blockIdx.x, n_items);
    const int t = threadIdx.x;
    const uint2 it = f.item_tab[item];
    const int tile = (int)it.x;
    s_cnt[t] = 0;
    const int px0 = (tile % f.ntx) * kTile, py0 = (tile / f.ntx) * kTile;
    const uint32_t lstart = f.tile_start[tile];
    const uint32_t n = f.tile_start[tile + 1] - lstart;
    const uint32_t j = it.y * kNT + t;
    SegRec s{};
    if (j < n) s = f.seg[f.list[lstart + j]];
    const uint32_t total = cov_setup(s, j < n, px0, py0, cam.W, cam.H, s_cov, s_own);
    wave_coverage(s_cov, s_own, total, [&](int p, int, int, int) { atomicAdd(&s_cnt[p], 1u); });
    __syncthreads();
    const size_t q = (size_t)tile * kTilePix + t;
    uint32_t base = 0;
    if (s_cnt[t]) base = atomicAdd(&f.pix_cnt[q], s_cnt[t]);
    f.item_base[(size_t)item * kTilePix + t] = base;
    PHASE_END(f.ctr, 0);
}

// Greedy batch packing of whole pixels: from p0 skip empty pixels, then take the longest run
// [p0, p1) whose fragments fit one LDS batch; a pixel deeper than a batch is "oversized" and
// forms a batch of its own.  Every lane finds, in parallel, the next non-empty pixel at or
// after it and the end of a batch that would start at it; the chain of batch starts is then
// followed (by one lane when it is short, by pointer doubling over all lanes when it is long)
// and marked in a 256-bit mask of the tile.  k_batch_records turns the mask
// into the batch table in parallel (a batch runs to the next start, or to the tile's end: the
// pixels in between are empty).
__global__ __launch_bounds__(kNT) void k_tile_prep(FrameBufs f) {
    __shared__ uint32_t s_cnt[kTilePix], s_off[kTilePix + 1], s_tmp[kNT];
    __shared__ uint16_t s_nxt[kTilePix + 1], s_end[kTilePix], s_jump[kTilePix + 1];
    __shared__ uint8_t s_on[kTilePix + 1];
    __shared__ uint32_t s_mask[kTilePix / 32];
    const int tile = blockIdx.x, t = threadIdx.x;
    const size_t q = (size_t)tile * kTilePix + t;
    const uint32_t c = f.pix_cnt[q];
    s_cnt[t] = c;
    uint32_t ex;
    const uint32_t total = block_exscan_u32(c, s_tmp, ex);
    s_off[t] = ex;
    f.pix_off[q] = ex;
    if (t == 0) s_off[kTilePix] = total;
    if (t < kTilePix / 32) s_mask[t] = 0u;
    __syncthreads();
    {   // next non-empty pixel q >= t: the smallest q with s_off[q + 1] > s_off[t]
        int lo = t, hi = kTilePix;
        const uint32_t o = s_off[t];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid + 1] > o) hi = mid; else lo = mid + 1;
        }
        s_nxt[t] = (uint16_t)lo;
    }
    if (c > (uint32_t)kCap) {
        s_end[t] = (uint16_t)(t + 1);
    } else {   // the largest p1 with s_off[p1] - s_off[t] <= kCap
        int lo = t + 1, hi = kTilePix;
        const uint32_t o0 = s_off[t];
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] - o0 <= (uint32_t)kCap) lo = mid; else hi = mid - 1;
        }
        s_end[t] = (uint16_t)lo;
    }
    if (t == 0) s_nxt[kTilePix] = (uint16_t)kTilePix;
    __syncthreads();
    if (total <= 16u * kCap) {   // a short chain (at most ~32 batches): one lane follows it
        if (t == 0) {
            uint32_t nb = 0, over = 0;
            for (int p = s_nxt[0]; p < kTilePix; p = s_nxt[s_end[p]]) {
                s_mask[p >> 5] |= 1u << (p & 31);
                ++nb;
                over += s_cnt[p] > (uint32_t)kCap;
            }
            f.tile_tot[tile] = total;
            f.tile_nb[tile] = nb;
            if (over) atomicAdd(&f.ctr->deep_pixels, over);
        }
    } else {
        // a long chain: every pixel marks where its batch's successor starts, and the marks
        // spread from the first start by pointer doubling (after step k, every start within
        // 2^(k+1) batches of the first; a tile has at most kTilePix = 2^8 batches).  A mark
        // seen early only spreads further along the same chain.
        s_jump[t] = s_nxt[s_end[t]];
        s_on[t] = 0;
        if (t == 0) {
            s_jump[kTilePix] = (uint16_t)kTilePix;
            s_on[kTilePix] = 0;
        }
        __syncthreads();
        if (t == 0) s_on[s_nxt[0]] = 1;
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            const int j = s_jump[t];
            if (s_on[t]) s_on[j] = 1;
            const uint16_t jj = s_jump[j];
            __syncthreads();
            s_jump[t] = jj;
            __syncthreads();
        }
        const bool on = s_on[t] != 0;
        const unsigned long long bm = __ballot(on), om = __ballot(on && c > (uint32_t)kCap);
        if ((t & 63) == 0) {
            s_mask[t >> 5] = (uint32_t)bm;
            s_mask[(t >> 5) + 1] = (uint32_t)(bm >> 32);
            s_tmp[t >> 6] = (uint32_t)__popcll(bm) | (uint32_t)__popcll(om) << 16;
        }
        __syncthreads();
        if (t == 0) {
            uint32_t nb = 0, over = 0;
            for (int w2 = 0; w2 < kNT / 64; ++w2) {
                nb += s_tmp[w2] & 0xFFFFu;
                over += s_tmp[w2] >> 16;
            }
            f.tile_tot[tile] = total;
            f.tile_nb[tile] = nb;
            if (over) atomicAdd(&f.ctr->deep_pixels, over);
        }
    }
    __syncthreads();
    if (t < kTilePix / 32) f.batch_mask[(size_t)tile * (kTilePix / 32) + t] = s_mask[t];
}

// The batch table: one record (tile, first pixel, end pixel, oversized) per marked start, in
// pixel order, at the tile's batch offset.
__global__ __launch_bounds__(kNT) void k_batch_records(FrameBufs f) {
    __shared__ uint32_t s_mask[kTilePix / 32], s_thk[kTilePix / 32];
    if (f.ctr->cap_overflow) return;
    const int tile = blockIdx.x, t = threadIdx.x;
    if (t < kTilePix / 32) s_mask[t] = f.batch_mask[(size_t)tile * (kTilePix / 32) + t];
    // (mixed frames: which pixels hold a thick-hair fragment, as bits)
    const unsigned long long tb = __ballot(f.pix_thick && f.pix_thick[(size_t)tile * kTilePix + t] != 0);
    if ((t & 63) == 0) {
        s_thk[t >> 5] = (uint32_t)tb;
        s_thk[(t >> 5) + 1] = (uint32_t)(tb >> 32);
    }
    __syncthreads();
    const int w = t >> 5, b = t & 31;
    if (!((s_mask[w] >> b) & 1u)) return;
    uint32_t idx = __popc(s_mask[w] & ((1u << b) - 1u));
    for (int k = 0; k < w; ++k) idx += __popc(s_mask[k]);
    int end = kTilePix;
    const uint32_t above = b == 31 ? 0u : (s_mask[w] >> (b + 1));
    if (above) {
        end = t + 1 + __ffs(above) - 1;
    } else {
        for (int k = w + 1; k < kTilePix / 32; ++k)
            if (s_mask[k]) {
                end = 32 * k + __ffs(s_mask[k]) - 1;
                break;
            }
    }
    const size_t tq = (size_t)tile * kTilePix;
    const bool oversized = f.pix_cnt[tq + t] > (uint32_t)kCap;
    const uint32_t off0 = f.pix_off[tq + t];
    const uint32_t off1 = end < kTilePix ? f.pix_off[tq + end] : f.tile_tot[tile];
    bool thick = false;   // a thick-hair fragment in pixels [t, end)
    for (int k = w; k <= (end - 1) >> 5; ++k) {
        uint32_t m = s_thk[k];
        if (k == w) m &= ~((1u << b) - 1u);
        if (k == (end - 1) >> 5 && ((end - 1) & 31) != 31) m &= (2u << ((end - 1) & 31)) - 1u;
        thick |= m != 0u;
    }
    const uint32_t pos = xcd_block_of(f.batch_start[tile] + idx, f.batch_start[f.T]);
    f.batches[pos] = pack_batch(tile, t, end, oversized, f.frag_base[tile] + off0, off1 - off0, thick);
    if (thick) f.thick_list[atomicAdd(&f.ctr->thick_batches, 1u)] = pos;
}

// Emit pass: every fragment into the frame's fragment buffer at
// frag_base[tile] + pix_off[pixel] + (the item's slice of the pixel) + local slot, and each
// pixel's depth-key range (LDS-aggregated per item).
// MIXED: a mixed-level frame, whose thick-hair pixels are marked in f.pix_thick.
template <bool MIXED>
__global__ __launch_bounds__(kNT) void k_emit(FrameBufs f, CamConst cam) {
    __shared__ uint32_t s_cur[kTilePix], s_pos[kTilePix], s_kmin[kTilePix], s_kmax[kTilePix];
    __shared__ uint32_t s_id[kNT];   // each owner's record word: global segment id or list index,
                                     // bit 31: a thick hair of a mixed frame
    __shared__ uint8_t s_thk[kTilePix];   // mixed frames: the pixel holds a thick-hair fragment
    __shared__ CovSetup s_cov[kNT];
    __shared__ uint8_t s_own[kNT / 64 * kCovLinesPerWave];
    __shared__ float2 s_iz[kNT];
    PHASE_BEGIN();
    const uint32_t n_items = f.item_start[f.T];
    if (blockIdx.x >= n_items || f.ctr->cap_overflow) return;
    const uint32_t item = xcd_contiguous(blockIdx.x, n_items);
    const int t = threadIdx.x;
    const uint2 it = f.item_tab[item];
    const int tile = (int)it.x;
    const size_t q = (size_t)tile * kTilePix + t;
    s_cur[t] = 0;
    s_kmin[t] = 0xFFFFFFFFu;
    s_kmax[t] = 0;
    s_thk[t] = 0;
    s_pos[t] = f.frag_base[tile] + f.pix_off[q] + f.item_base[(size_t)item * kTilePix + t];
    __syncthreads();
    const int px0 = (tile % f.ntx) * kTile, py0 = (tile / f.ntx) * kTile;
    const uint32_t lstart = f.tile_start[tile];
    const uint32_t n = f.tile_start[tile + 1] - lstart;
    const uint32_t j = it.y * kNT + t;
    SegRec s{};
    uint32_t gseg = 0;
    if (j < n) {
        gseg = f.list[lstart + j];
        s = f.seg[gseg];
    }
    s_iz[t] = make_float2(s.iza, s.izb);
    s_id[t] = (f.gid ? gseg : j) | (MIXED && (s.hwfx & kFlagThick) ? 0x80000000u : 0u);
    const uint32_t total = cov_setup(s, j < n, px0, py0, cam.W, cam.H, s_cov, s_own);
    wave_coverage(s_cov, s_own, total, [&](int p, int tnum, int tden, int o) {
        const float2 iz = s_iz[o];
        const uint32_t key = depth_key_iz(iz.x, iz.y, tnum, tden);
        const uint32_t slot = atomicAdd(&s_cur[p], 1u);
        atomicMin(&s_kmin[p], key);
        atomicMax(&s_kmax[p], key);
        const uint32_t id = s_id[o];
        if (MIXED && (id >> 31)) s_thk[p] = 1;
        f.frags[s_pos[p] + slot] = make_uint2(key, (id & 0xFFFFFFu) | ((uint32_t)p << 24));
    });
    __syncthreads();
    if (s_cur[t]) {
        atomicMin(&f.pix_kmin[q], s_kmin[t]);
        atomicMax(&f.pix_kmax[q], s_kmax[t]);
        if (MIXED && s_thk[t]) f.pix_thick[q] = 1;
    }
    PHASE_END(f.ctr, 1);
}

// The bucket map's scale of a pixel of cnt records with keys in [kmin, kmax].
__device__ inline float bucket_scale(uint32_t cnt, uint32_t kmin, uint32_t kmax) {
    return (float)cnt * __builtin_amdgcn_rcpf((float)(kmax - kmin) + 1.0f);
}

// Exact per-pixel order of the Fb records rec (records i = t + qq kNT; entries beyond Fb are
// ignored) of whole pixels with counts, key minima, bucket scales and offsets in s_cnt /
// s_kmin / s_scale / s_off, into s_B.  Bucket sort with one bucket per record, bucket = the
// record's place in its pixel's linear key range (s_scale[p] = count / (key range + 1): a
// monotone map, so sorted buckets give a sorted pixel); the records are scattered to bucket
// order in s_A, and each record's place inside its bucket is its rank there by (key, segment
// id), which is unique within a pixel.  A thread's LDS reads of one step are issued together,
// and a bucket of up to four records is ranked from one set of reads (larger ones loop).
// s_bk must hold Fb zeros on entry.  Ends with a barrier.
__device__ inline void order_batch(uint32_t Fb, const uint2 (&rec)[kPerThread], const uint32_t* s_cnt,
                                   const uint32_t* s_kmin, const float* s_scale, const uint32_t* s_off,
                                   uint32_t* s_tmp, uint2* s_A, uint2* s_B, uint32_t* s_bk, const uint32_t* list,
                                   bool gid) {
    const int t = threadIdx.x;
    uint32_t my_b[kPerThread], my_r[kPerThread];
    {
        uint32_t kmn[kPerThread], cnt[kPerThread], off[kPerThread];
        float sc[kPerThread];
#pragma unroll
        for (int qq = 0; qq < kPerThread; ++qq) {
            const uint32_t p = rec[qq].y >> 24;   // (< 256 for any record)
            kmn[qq] = s_kmin[p];
            sc[qq] = s_scale[p];
            off[qq] = s_off[p];
            cnt[qq] = s_cnt[p];
        }
#pragma unroll
        for (int qq = 0; qq < kPerThread; ++qq)
            my_b[qq] = off[qq] + min(cnt[qq] - 1u, (uint32_t)((float)(rec[qq].x - kmn[qq]) * sc[qq]));
#pragma unroll
        for (int qq = 0; qq < kPerThread; ++qq)
            if (t + qq * kNT < Fb) my_r[qq] = atomicAdd(&s_bk[my_b[qq]], 1u);
    }
    __syncthreads();
    {   // exclusive scan of the bucket counters, kOwn consecutive per thread (odd, so the
        // lanes' strided reads fall in distinct LDS banks)
        constexpr int kOwn = kPerThread + 1;
        uint32_t loc[kOwn];
        uint32_t sum = 0;
#pragma unroll
        for (int qq = 0; qq < kOwn; ++qq) {
            const uint32_t i = t * kOwn + qq;
            loc[qq] = i < Fb ? s_bk[i] : 0u;
            sum += loc[qq];
        }
        uint32_t ex;
        block_exscan_u32(sum, s_tmp, ex);
#pragma unroll
        for (int qq = 0; qq < kOwn; ++qq) {
            const uint32_t i = t * kOwn + qq;
            if (i < Fb) s_bk[i] = ex;
            ex += loc[qq];
        }
    }
    __syncthreads();
    uint32_t b0[kPerThread], b1[kPerThread];
#pragma unroll
    for (int qq = 0; qq < kPerThread; ++qq) {
        const bool ok = t + qq * kNT < Fb;
        b0[qq] = ok ? s_bk[my_b[qq]] : 0u;
        b1[qq] = ok && my_b[qq] + 1 < Fb ? s_bk[my_b[qq] + 1] : Fb;
    }
#pragma unroll
    for (int qq = 0; qq < kPerThread; ++qq)
        if (t + qq * kNT < Fb) s_A[b0[qq] + my_r[qq]] = rec[qq];
    __syncthreads();
    // ranks, two records at a time (each one's bucket read with independent loads)
    constexpr uint32_t kSmall = 4;
    static_assert(kPerThread % 2 == 0, "records are ranked in pairs");
#pragma unroll
    for (int q0 = 0; q0 < kPerThread; q0 += 2) {
        uint2 u[2][kSmall];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int qq = q0 + h;
            const uint32_t n = t + qq * kNT < Fb ? b1[qq] - b0[qq] : 1u;
#pragma unroll
            for (uint32_t k = 0; k < kSmall; ++k) u[h][k] = n > 1 ? s_A[b0[qq] + min(k, n - 1)] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int qq = q0 + h;
            if (t + qq * kNT >= Fb) continue;
            const uint2 me = rec[qq];
            const uint32_t n = b1[qq] - b0[qq];
            uint32_t rank = 0;
            auto before = [&](const uint2& v) {   // (key, segment id) of v below me's
                bool less = v.x < me.x;
                if (v.x == me.x) less = seg_of(v.y, list, gid) < seg_of(me.y, list, gid);
                return less;
            };
#pragma unroll
            for (uint32_t k = 0; k < kSmall; ++k)
                if (k < n && k != my_r[qq]) rank += before(u[h][k]);
            for (uint32_t k = kSmall; k < n; ++k)
                if (k != my_r[qq]) rank += before(s_A[b0[qq] + k]);
            s_B[b0[qq] + rank] = me;
        }
    }
    __syncthreads();
}

// The backward pass's ordering: the same buckets, records staged in s_A and sorted in place in
// s_B by insertion inside each bucket.  (The rank-based routine above gives the same order, but
// inside k_batch_bwd, whose registers are at the 256 + AGPR limit, its use changes that
// kernel's gradients; this variant is the one validated there.)  s_bk must hold Fb zeros.
__device__ inline void order_batch_insertion(uint32_t Fb, const uint32_t* s_cnt, const uint32_t* s_kmin,
                                             const uint32_t* s_kmax, const uint32_t* s_off, uint32_t* s_tmp,
                                             const uint2* s_A, uint2* s_B, uint32_t* s_bk, const uint32_t* list) {
    const int t = threadIdx.x;
    uint32_t my_b[kPerThread], my_r[kPerThread];
#pragma unroll
    for (int qq = 0; qq < kPerThread; ++qq) {
        const uint32_t i = t + qq * kNT;
        if (i < Fb) {
            const uint2 rec = s_A[i];
            const uint32_t p = rec.y >> 24;
            const uint32_t kmn = s_kmin[p], cnt = s_cnt[p];
            const float scale = (float)cnt * __builtin_amdgcn_rcpf((float)(s_kmax[p] - kmn) + 1.0f);
            const uint32_t bucket = min(cnt - 1u, (uint32_t)((float)(rec.x - kmn) * scale));
            my_b[qq] = s_off[p] + bucket;
            my_r[qq] = atomicAdd(&s_bk[my_b[qq]], 1u);
        }
    }
    __syncthreads();
    {
        uint32_t loc[kPerThread];
        uint32_t sum = 0;
#pragma unroll
        for (int qq = 0; qq < kPerThread; ++qq) {
            const uint32_t i = t * kPerThread + qq;
            loc[qq] = i < Fb ? s_bk[i] : 0u;
            sum += loc[qq];
        }
        uint32_t ex;
        block_exscan_u32(sum, s_tmp, ex);
#pragma unroll
        for (int qq = 0; qq < kPerThread; ++qq) {
            const uint32_t i = t * kPerThread + qq;
            if (i < Fb) s_bk[i] = ex;
            ex += loc[qq];
        }
    }
    __syncthreads();
#pragma unroll
    for (int qq = 0; qq < kPerThread; ++qq) {
        const uint32_t i = t + qq * kNT;
        if (i < Fb) s_B[s_bk[my_b[qq]] + my_r[qq]] = s_A[i];
    }
    __syncthreads();
    for (uint32_t bi = t; bi < Fb; bi += kNT) {
        const uint32_t b0 = s_bk[bi];
        const uint32_t b1 = bi + 1 < Fb ? s_bk[bi + 1] : Fb;
        for (uint32_t i = b0 + 1; i < b1; ++i) {
            const uint2 v = s_B[i];
            const uint32_t vseg = list[v.y & 0xFFFFFFu];
            uint32_t jx = i;
            while (jx > b0) {
                const uint2 u2 = s_B[jx - 1];
                bool greater = u2.x > v.x;
                if (u2.x == v.x) greater = list[u2.y & 0xFFFFFFu] > vseg;
                if (!greater) break;
                s_B[jx] = u2;
                --jx;
            }
            s_B[jx] = v;
        }
    }
    __syncthreads();
}

// LDS working set of one batch.
struct BatchLds {
    uint32_t* s_cnt;
    uint32_t* s_kmin;
    float* s_scale;
    uint32_t* s_off;
    uint32_t* s_tmp;
    uint2* s_B;
    uint2* s_A;
    uint32_t* s_bk;
    float* s_agg;
    uint32_t* s_aggh;
};

// Exact order, shading and blending of the Fb records staged in s_A (whole pixels whose
// counts, key minima, bucket scales and offsets are in s_cnt / s_kmin / s_scale / s_off).  Finished pixels are
// written to rgba, or (slice_out != nullptr, a single pixel's key slice) their (C, T) goes to
// slice_out.  rank0 / cnt_total place a slice inside its pixel for the debug dump; by_seg: the
// records carry segment ids in place of keys (a slice inside one key, key_of_slice).
template <int KIND, int MODEL, bool SHADOW>
__device__ inline void sort_shade_blend(const FrameBufs& f, const ShadeArgs& a, float* __restrict__ rgba,
                                        const DebugDump& dbg, int has_dbg, const BatchLds& L_, const uint32_t* list,
                                        const uint2 (&rec)[kPerThread], int px0, int py0, uint32_t Fb, float* slice_out,
                                        uint32_t rank0, uint32_t cnt_total, bool by_seg = false,
                                        uint32_t key_of_slice = 0u) {
    uint32_t* s_cnt = L_.s_cnt;
    uint32_t* s_kmin = L_.s_kmin;
    const float* s_scale = L_.s_scale;
    uint32_t* s_off = L_.s_off;
    uint32_t* s_tmp = L_.s_tmp;
    uint2* s_B = L_.s_B;
    uint2* s_A = L_.s_A;
    uint32_t* s_bk = L_.s_bk;
    float* s_agg = L_.s_agg;
    uint32_t* s_aggh = L_.s_aggh;
    const int t = threadIdx.x;
    const int W = a.cam.W, H = a.cam.H;
    PHASE_BEGIN();
    const bool gid = f.gid != 0;
    order_batch(Fb, rec, s_cnt, s_kmin, s_scale, s_off, s_tmp, s_A, s_B, s_bk, list, gid);
    PHASE_END(f.ctr, 2);
    // ---- shade and blend: thread t takes the run [rb, re) of consecutive fragments of the
    // ordered batch, shades them in order and composites them front to back ("over") as it
    // goes, restarting at each pixel's first fragment.  A pixel that begins and ends inside
    // the run is finished there; the run's first pixel, when it began in an earlier run, is
    // finished after a segmented scan of the runs' open composites gives what lies in front.
    // The segment ids of a thread's fragments are gathered up front (independent loads) and
    // each fragment's segment inputs are fetched one fragment ahead, so that the gathers
    // overlap the shading arithmetic.  (Not for the R / TT / TRT thick-hair shading: its
    // registers would then exceed the budget of three waves per SIMD.)
    constexpr bool kAhead = KIND == 0 || KIND == 3 || (KIND == 1 && MODEL == 1);
    const uint32_t run = (Fb + kNT - 1) / kNT;   // at most kPerThread
    const uint32_t rb = min(Fb, t * run), re = min(Fb, rb + run);
    // Mixed frames shade before they blend: a wave whose lanes held both strand and thick-hair
    // fragments would run both shading paths in turn, so the batch's fragments are listed
    // strands first, thick hairs after, shaded kNT at a time down that list (only the wave at
    // the boundary holds both kinds), and each one's (alpha, L) is staged in LDS for the blend.
    // (Not with the debug dump, which also records h, nor in a batch of strands alone.)
    bool staged = false;
    float4* s_res = reinterpret_cast<float4*>(s_A);   // free once the batch is ordered
    if (KIND == 2 && !has_dbg) {
        uint16_t* s_lst = reinterpret_cast<uint16_t*>(reinterpret_cast<uint32_t*>(s_A) + 4 * kCap);
        uint32_t thick = 0, ns = 0;
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const uint32_t i = t + k * kNT;
            if (i < Fb) {
                if (a.seg[seg_of(s_B[i].y, list, gid)].hwfx & kFlagThick) thick |= 1u << k;
                else ++ns;
            }
        }
        uint32_t ex;
        const uint32_t tot = block_exscan_u32(ns | (uint32_t)__popc(thick) << 16, s_tmp, ex);
        const uint32_t n_s = tot & 0xFFFFu;
        staged = (tot >> 16) > 0;   // uniform across the block
        if (staged) {
            uint32_t ps = ex & 0xFFFFu, pt = n_s + (ex >> 16);
#pragma unroll
            for (int k = 0; k < kPerThread; ++k) {
                const uint32_t i = t + k * kNT;
                if (i < Fb) s_lst[((thick >> k) & 1u) ? pt++ : ps++] = (uint16_t)i;
            }
            __syncthreads();
            for (uint32_t jj = t; jj < Fb; jj += kNT) {
                const uint32_t i = s_lst[jj];
                const uint2 rec = s_B[i];
                const uint32_t p = rec.y >> 24;
                float al, hh, L[3];
                shade_inputs<KIND, MODEL, SHADOW>(a, fetch_segment<KIND>(a, seg_of(rec.y, list, gid)),
                                                  px0 + (int)(p % kTile), py0 + (int)(p / kTile), al, hh, L);
                s_res[i] = make_float4(al, L[0], L[1], L[2]);
            }
            __syncthreads();
        }
    }
    uint32_t gs[kAhead ? kPerThread : 1];
    SegInputs nxt{};
    if (kAhead) {
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            const uint32_t i = rb + j;
            gs[j] = i < re ? seg_of(s_B[i].y, list, gid) : 0u;
        }
        if (rb < re) nxt = fetch_segment<KIND>(a, gs[0]);
    }
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;   // the open pixel's composite so far
    uint32_t head = 0;                             // the open pixel began in this run
    float H0 = 0.f, H1 = 0.f, H2 = 0.f, HT = 1.f;  // the run's first pixel, begun earlier, ended here
    int hp = -1;
    auto finish = [&](int p, float c0, float c1, float c2, float tt) {
        if (slice_out) {
            slice_out[0] = c0; slice_out[1] = c1; slice_out[2] = c2; slice_out[3] = tt;
        } else {
            const int gx = px0 + (p % kTile), gy = py0 + (p / kTile);
            if (gx < W && gy < H) reinterpret_cast<float4*>(rgba)[(size_t)gy * W + gx] = make_float4(c0, c1, c2, 1.0f - tt);
        }
    };
    for (uint32_t i = rb; i < re; ++i) {
        SegInputs cur{};
        uint32_t gseg = 0;
        if (!(KIND == 2 && staged)) {   // (the next fragment's inputs are requested first)
            if (!kAhead) gs[0] = seg_of(s_B[i].y, list, gid);
            cur = kAhead ? nxt : fetch_segment<KIND>(a, gs[0]);
            gseg = gs[0];
            if (kAhead) {
#pragma unroll
                for (int j = 0; j + 1 < (kAhead ? kPerThread : 1); ++j) gs[j] = gs[j + 1];
                if (i + 1 < re) nxt = fetch_segment<KIND>(a, gs[0]);
            }
        }
        const uint2 rec = s_B[i];
        const uint32_t p = rec.y >> 24;
        const uint32_t p_beg = s_off[p], p_end = s_off[p + 1];
        if (i == p_beg) { C0 = C1 = C2 = 0.f; T = 1.f; head = 1; }
        const int gx = px0 + (int)(p % kTile), gy = py0 + (int)(p / kTile);
        float al, hh, L[3];
        if (KIND == 2 && staged) {
            const float4 r = s_res[i];
            al = r.x; L[0] = r.y; L[1] = r.z; L[2] = r.w;
            hh = 0.f;
        } else {
            shade_inputs<KIND, MODEL, SHADOW>(a, cur, gx, gy, al, hh, L);
        }
        C0 += T * (al * L[0]);
        C1 += T * (al * L[1]);
        C2 += T * (al * L[2]);
        T *= 1.0f - al;
        if (i + 1 == p_end) {
            if (head) finish((int)p, C0, C1, C2, T);
            else { H0 = C0; H1 = C1; H2 = C2; HT = T; hp = (int)p; }
        }
        if (has_dbg) {
            const int dx = gx - dbg.x0, dy = gy - dbg.y0;
            if (dx >= 0 && dy >= 0 && dx < dbg.w && dy < dbg.h) {
                const uint32_t rank = i - p_beg + rank0;
                const int q2 = dy * dbg.w + dx;
                if (rank == 0) dbg.counts[q2] = cnt_total ? cnt_total : s_cnt[p];
                if ((int)rank < dbg.stride) {
                    const size_t o = (size_t)q2 * dbg.stride + rank;
                    dbg.keys[o] = by_seg ? key_of_slice : rec.x;
                    dbg.segs[o] = gseg;
                    dbg.alpha[o] = al;
                    dbg.hoff[o] = hh;
                }
            }
        }
    }
    PHASE_END(f.ctr, 3);
    // inclusive scan of the runs' open composites, (l) then (r) = r.head ? r : (l.C + l.T r.C,
    // l.T r.T): within the wave by shuffles, then across the block's waves through LDS; a thread
    // with no fragments passes its left neighbour's composite through
    const int lane = t & 63, wv = t >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const float c0 = __shfl_up(C0, off), c1 = __shfl_up(C1, off), c2 = __shfl_up(C2, off);
        const float tt = __shfl_up(T, off);
        const uint32_t hh2 = __shfl_up(head, off);
        if (lane >= off && !head) {
            C0 = c0 + tt * C0;
            C1 = c1 + tt * C1;
            C2 = c2 + tt * C2;
            T = tt * T;
            head = hh2;
        }
    }
    const float l0 = __shfl_up(C0, 1), l1 = __shfl_up(C1, 1), l2 = __shfl_up(C2, 1), lT = __shfl_up(T, 1);
    const uint32_t lh = __shfl_up(head, 1);
    if (lane == 63) {
        s_agg[4 * wv + 0] = C0; s_agg[4 * wv + 1] = C1; s_agg[4 * wv + 2] = C2; s_agg[4 * wv + 3] = T;
        s_aggh[wv] = head;
    }
    __syncthreads();
    if (hp >= 0) {   // what lies in front of this run: earlier waves, then earlier lanes of this wave
        float e0 = 0.f, e1 = 0.f, e2 = 0.f, eT = 1.f;
        for (int w2 = 0; w2 < wv; ++w2) {
            if (s_aggh[w2]) { e0 = s_agg[4 * w2 + 0]; e1 = s_agg[4 * w2 + 1]; e2 = s_agg[4 * w2 + 2]; eT = s_agg[4 * w2 + 3]; }
            else {
                e0 = e0 + eT * s_agg[4 * w2 + 0];
                e1 = e1 + eT * s_agg[4 * w2 + 1];
                e2 = e2 + eT * s_agg[4 * w2 + 2];
                eT = eT * s_agg[4 * w2 + 3];
            }
        }
        if (lane > 0) {
            if (lh) { e0 = l0; e1 = l1; e2 = l2; eT = lT; }
            else {
                e0 = e0 + eT * l0;
                e1 = e1 + eT * l1;
                e2 = e2 + eT * l2;
                eT = eT * lT;
            }
        }
        finish(hp, e0 + eT * H0, e1 + eT * H1, e2 + eT * H2, eT * HT);
    }
    PHASE_END(f.ctr, 4);
}

// Slice of a deep pixel's k records at src: among the records that val(r, v) admits, with
// value v in [lo, end), the longest run of leading histogram bins holding at most kCap of them
// (bins refined until one fits).  Returns 0 with [lo, *hi) and its record count *Fb, or 2 when
// more than kCap admitted records share the single value lo.  Values are 32-bit, so lo < 2^32,
// the bin width stays below 2^22 and bins are exact 32-bit quotients.  s_bk holds the
// histogram (kCap bins); all threads call it; ends with a barrier.
template <class Val>
__device__ inline uint32_t refine_slice(uint32_t k, const uint2* __restrict__ src, unsigned long long lo,
                                        unsigned long long end, Val&& val, uint32_t* s_bk, uint32_t* s_tmp,
                                        unsigned long long* s_range, uint32_t& s_slot, uint32_t& s_flag,
                                        unsigned long long& hi_out, uint32_t& Fb) {
    constexpr uint32_t kBins = kCap;
    const int t = threadIdx.x;
    unsigned long long range_hi = end;
    while (true) {
        const unsigned long long width = (range_hi - lo + kBins - 1) / kBins;
        const uint32_t lo32 = (uint32_t)lo, w32 = (uint32_t)width;
        for (uint32_t i = t; i < kBins; i += kNT) s_bk[i] = 0;
        __syncthreads();
        // histogram of the admitted values in [lo, range_hi); each lane's loads issued together
        for (uint32_t i0 = 0; i0 < k; i0 += kNT * kPerThread) {
            uint2 rr[kPerThread];
#pragma unroll
            for (int qq = 0; qq < kPerThread; ++qq) {
                const uint32_t i = i0 + t + qq * kNT;
                rr[qq] = i < k ? src[i] : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int qq = 0; qq < kPerThread; ++qq) {
                const uint32_t i = i0 + t + qq * kNT;
                uint32_t v;
                if (i < k && val(rr[qq], v) && v >= lo32 && (unsigned long long)v < range_hi)
                    atomicAdd(&s_bk[(v - lo32) / w32], 1u);
            }
        }
        __syncthreads();
        // the longest run of leading bins holding at most kCap records, from a block scan of the
        // bin counts (lane t owns bins t * kPerThread ...): the one lane that owns the run's last
        // bin writes the slice; lane 0 flags a first bin that alone exceeds kCap
        {
            const uint32_t used = (uint32_t)((range_hi - lo + width - 1) / width);
            uint32_t loc[kPerThread], sum = 0;
#pragma unroll
            for (int qq = 0; qq < kPerThread; ++qq) {
                const uint32_t i = t * kPerThread + qq;
                loc[qq] = i < used ? s_bk[i] : 0u;
                sum += loc[qq];
            }
            uint32_t incl;
            block_exscan_u32(sum, s_tmp, incl);
#pragma unroll
            for (int qq = 0; qq < kPerThread; ++qq) {
                const uint32_t i = t * kPerThread + qq;
                incl += loc[qq];
                if (i < used && incl <= (uint32_t)kCap) {
                    const uint32_t nxt = i + 1 >= used ? 0u : (qq + 1 < kPerThread ? loc[qq + 1] : s_bk[i + 1]);
                    if (i + 1 >= used || incl + nxt > (uint32_t)kCap) {
                        s_flag = 0;
                        s_range[1] = min(range_hi, lo + (unsigned long long)(i + 1) * width);
                        s_slot = incl;
                    }
                }
            }
            if (t == 0 && loc[0] > (uint32_t)kCap) {
                s_flag = width == 1 ? 2u : 1u;     // 1: refine inside the first bin; 2: one value overflows
                s_range[1] = lo + width;
            }
        }
        __syncthreads();
        const uint32_t flag = s_flag;
        range_hi = s_range[1];
        Fb = s_slot;
        __syncthreads();
        if (flag != 1) {
            hi_out = range_hi;
            return flag;
        }
    }
}

// One LDS batch of whole pixels: exact per-pixel order, shading, front-to-back blending.  A
// pixel deeper than one batch (its own "oversized" batch) is processed in depth-key slices:
// a histogram over the pixel's key range picks the longest run of bins that fits LDS, those
// records are gathered and processed exactly, and the slice composites chain front to back.
// (LDS holds four blocks per CU; unshadowed strand instances keep their registers within four waves
// per SIMD, the heavier shading (thick hairs, shadowed strands) within three.)
template <int KIND, int MODEL, bool SHADOW>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu((KIND == 0 || KIND == 3) && !SHADOW ? 4 : 3))) void k_batch(
    FrameBufs f, ShadeArgs a, float* __restrict__ rgba, DebugDump dbg, int has_dbg) {
    __shared__ uint32_t s_cnt[kTilePix], s_kmin[kTilePix], s_off[kTilePix + 1];
    __shared__ float s_scale[kTilePix];   // count / (key range + 1): the bucket map of the ordering
    __shared__ uint32_t s_tmp[kNT];
    __shared__ __align__(16) uint2 s_B[kCap];
    // staged records (2 words) + bucket counters; in mixed frames also, after the ordering, each
    // fragment's (alpha, L) and the batch's fragments listed strands first (kCap 16-bit entries)
    __shared__ __align__(16) uint32_t s_work[KIND == 2 ? 4 * kCap + kCap / 2 : 3 * kCap];
    __shared__ float s_agg[kNT / 64 * 4];     // wave aggregates of the blend scan (C rgb, T)
    __shared__ uint32_t s_aggh[kNT / 64];
    __shared__ float s_slice[4];
    __shared__ unsigned long long s_range[2];
    __shared__ uint32_t s_slot, s_flag;
    BatchLds L_{s_cnt, s_kmin, s_scale, s_off, s_tmp, s_B, reinterpret_cast<uint2*>(s_work), s_work + 2 * kCap, s_agg,
                s_aggh};
    PHASE_BEGIN();

    const uint32_t n_batches = f.batch_start[f.T];
    // Mixed frames take two launches.  When at most an eighth of the batches hold thick-hair
    // fragments, the strand-only kernel (KIND 3, four waves per SIMD) takes the batches of
    // strands alone and this one (KIND 2) those holding thick hairs, block b the b-th of their
    // list (spread over the grid, and so over the XCDs, wherever on screen the thick hairs lie).
    // Otherwise KIND 2 takes every batch, so that its long thick-hair batches interleave with
    // the rest, and KIND 3 does nothing.
    uint32_t bi = blockIdx.x;
    if (KIND == 2 || KIND == 3) {
        const bool one = f.thick_list == nullptr || 8u * f.ctr->thick_batches > n_batches;
        if (KIND == 3 && one) return;
        if (KIND == 2 && !one) {
            if (blockIdx.x >= f.ctr->thick_batches) return;
            bi = f.thick_list[blockIdx.x];
        }
    }
    const uint4 br = f.batches[bi];   // in the table's capacity; used only below n_batches
    if (bi >= n_batches || f.ctr->cap_overflow) return;
    const BatchRec b = unpack_batch(br);
    if (KIND == 3 && b.thick) return;
    const int tile = b.tile, p0 = b.p0, p1 = b.p1;
    const int t = threadIdx.x;
    const int px0 = (tile % f.ntx) * kTile, py0 = (tile / f.ntx) * kTile;
    const int W = a.cam.W, H = a.cam.H;
    const uint32_t* list = f.list + f.tile_start[tile];
    const size_t q = (size_t)tile * kTilePix + t;
    const uint2* src = f.frags + b.frag0;
    if (!b.over) {
        // the batch's records, its pixels' counts, key ranges and offsets: all loads in flight
        // together before the first barrier
        const uint32_t Fb = b.nfrag;
        uint2 rec[kPerThread];
#pragma unroll
        for (int qq = 0; qq < kPerThread; ++qq) {
            const uint32_t i = t + qq * kNT;
            rec[qq] = i < Fb ? src[i] : make_uint2(0u, 0u);
        }
        const uint32_t tile_off0 = f.pix_off[(size_t)tile * kTilePix + p0];
        if (t >= p0 && t < p1) {
            const uint32_t cnt = f.pix_cnt[q], kmn = f.pix_kmin[q];
            s_cnt[t] = cnt;
            s_kmin[t] = kmn;
            s_scale[t] = bucket_scale(cnt, kmn, f.pix_kmax[q]);
            s_off[t] = f.pix_off[q] - tile_off0;
        }
        if (t == 0) s_off[p1] = Fb;
        for (uint32_t i = t; i < Fb; i += kNT) L_.s_bk[i] = 0;
        __syncthreads();
        PHASE_END(f.ctr, 5);
        sort_shade_blend<KIND, MODEL, SHADOW>(f, a, rgba, dbg, has_dbg, L_, list, rec, px0, py0, Fb, nullptr, 0, 0);
        return;
    }
    // ---- a pixel deeper than one batch: exact slices in (key, segment id) order
    const int p = p0;
    const size_t qp = (size_t)tile * kTilePix + p;
    const uint32_t k = b.nfrag;
    const unsigned long long key_end = (unsigned long long)f.pix_kmax[qp] + 1ull;
    unsigned long long lo = f.pix_kmin[qp];
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;   // carried composite (thread 0)
    uint32_t done = 0;
    PHASE_ADD(f.ctr, 7, k);
    PHASE_END(f.ctr, 5);
    // one slice: the records whose value (their key, or inside one key their segment id) lies
    // in [v_lo, v_hi), staged as (value, local index | pixel), ordered, shaded and blended
    auto run_slice = [&](uint32_t Fb, unsigned long long v_lo, unsigned long long v_hi, auto&& val, bool by_seg,
                         uint32_t key) {
        if (t == 0) s_slot = 0;
        __syncthreads();
        for (uint32_t i0 = 0; i0 < k; i0 += kNT * kPerThread) {
            uint2 rr[kPerThread];
#pragma unroll
            for (int qq = 0; qq < kPerThread; ++qq) {
                const uint32_t i = i0 + t + qq * kNT;
                rr[qq] = i < k ? src[i] : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int qq = 0; qq < kPerThread; ++qq) {
                const uint32_t i = i0 + t + qq * kNT;
                uint32_t v;
                if (i < k && val(rr[qq], v) && (unsigned long long)v >= v_lo && (unsigned long long)v < v_hi)
                    L_.s_A[atomicAdd(&s_slot, 1u)] = make_uint2(v, rr[qq].y);
            }
        }
        __syncthreads();
        for (uint32_t i = t; i < Fb; i += kNT) L_.s_bk[i] = 0;
        if (t == 0) {
            s_cnt[p] = Fb;
            s_kmin[p] = (uint32_t)v_lo;
            s_scale[p] = bucket_scale(Fb, (uint32_t)v_lo, (uint32_t)(v_hi - 1));
            s_off[p] = 0;
            s_off[p + 1] = Fb;
        }
        __syncthreads();
        PHASE_END(f.ctr, 6);
        uint2 rec[kPerThread];
#pragma unroll
        for (int qq = 0; qq < kPerThread; ++qq) {
            const uint32_t i = t + qq * kNT;
            rec[qq] = i < Fb ? L_.s_A[i] : make_uint2(0u, 0u);
        }
        sort_shade_blend<KIND, MODEL, SHADOW>(f, a, rgba, dbg, has_dbg, L_, list, rec, px0, py0, Fb, s_slice, done, k,
                                              by_seg, key);
        PHASE_RESET();
        __syncthreads();
        if (t == 0) {
            C0 += T * s_slice[0];
            C1 += T * s_slice[1];
            C2 += T * s_slice[2];
            T *= s_slice[3];
        }
        done += Fb;
        __syncthreads();
    };
    auto by_key = [&](const uint2& r, uint32_t& v) { v = r.x; return true; };
    while (lo < key_end) {
        unsigned long long hi;
        uint32_t Fb;
        const uint32_t flag = refine_slice(k, src, lo, key_end, by_key, L_.s_bk, s_tmp, s_range, s_slot, s_flag, hi, Fb);
        if (flag == 0) {
            // (a slice of leading empty bins holds no record and changes nothing)
            if (Fb) run_slice(Fb, lo, hi, by_key, false, 0u);
            lo = hi;
            continue;
        }
        // more than one batch of fragments at one key K0: slices by segment id inside it (a
        // segment meets a pixel once, so every id range refines down to a slice that fits)
        const uint32_t K0 = (uint32_t)lo;
        auto by_seg = [&](const uint2& r, uint32_t& v) {
            if (r.x != K0) return false;
            v = seg_of(r.y, list, f.gid != 0);
            return true;
        };
        unsigned long long slo = 0;
        const unsigned long long send = 1ull << 32;
        while (slo < send) {
            unsigned long long shi;
            if (refine_slice(k, src, slo, send, by_seg, L_.s_bk, s_tmp, s_range, s_slot, s_flag, shi, Fb) != 0) {
                if (t == 0) atomicAdd(&f.ctr->overflow_pixels, 1u);   // (not reachable: ids are unique)
                return;
            }
            if (Fb) run_slice(Fb, slo, shi, by_seg, true, K0);
            slo = shi;
        }
        lo = (unsigned long long)K0 + 1ull;
    }
    if (t == 0) {
        const int gx = px0 + (p % kTile), gy = py0 + (p / kTile);
        if (gx < W && gy < H) reinterpret_cast<float4*>(rgba)[(size_t)gy * W + gx] = make_float4(C0, C1, C2, 1.0f - T);
    }
}

// ---------------------------------------------------------------------------------------
// Backward pass (thick-hair levels): vector-Jacobian product of the frame with respect to
// each cluster segment's |a|, |b| and its cluster's r and sigma_a.  Per batch:
//   1. the forward's exact per-pixel order (same bucket sort);
//   2. alpha_k and L_k per fragment (float);
//   3. front-to-back prefix T_k and back-to-front suffix (C_k+, S_k+) by two segmented scans;
//      with dC, dA the pixel's output adjoint:
//        dLoss/dalpha_k = T_k [dC . (L_k - C_k+) + dA S_k+],   dLoss/dL_k = dC T_k alpha_k;
//   4. alpha_k and L_k again as Dual<6> (forward-mode partials in |a|, |b|, r, sigma_a rgb)
//      contracted with the step-3 adjoints; partials summed per list entry in LDS, then one
//      global atomic per (batch, list entry, parameter).
constexpr int kNAcc = 1024;          // list entries with LDS accumulators (others go straight to global)
using Dual6 = Dual<6>;

// d hw / d|a|, d hw / d|b| of the float32 half-width (support of the ellipse across the view at
// the segment midpoint, times fy / z_mid).
__device__ inline void halfwidth_partials(const CamConst& c, const SegRec& s, const float4& q0, const float4& q1,
                                          const float4& q2, float a_len, float b_len, float& da, float& db) {
    const float tx = q1.x - q0.x, ty = q1.y - q0.y, tz = q1.z - q0.z;
    const float tl = norm3f(tx, ty, tz);
    const float ux = tx / tl, uy = ty / tl, uz = tz / tl;
    const float mx = (q0.x + q1.x) * 0.5f, my = (q0.y + q1.y) * 0.5f, mz = (q0.z + q1.z) * 0.5f;
    float wx = c.pos[0] - mx, wy = c.pos[1] - my, wz = c.pos[2] - mz;
    const float wl = norm3f(wx, wy, wz);
    wx /= wl; wy /= wl; wz /= wl;
    const float dwu = (wx * ux + wy * uy) + wz * uz;
    const float px = wx - dwu * ux, py = wy - dwu * uy, pz = wz - dwu * uz;
    const float pl = norm3f(px, py, pz);
    const float zm = (1.0f / s.iza + 1.0f / s.izb) * 0.5f;
    const float k = c.fy / zm;
    if (!(pl > 1e-7f)) {
        da = a_len >= b_len ? k : 0.0f;
        db = a_len >= b_len ? 0.0f : k;
        return;
    }
    const float xx = px / pl, xy = py / pl, xz = pz / pl;
    const float yx = uy * xz - uz * xy, yy = uz * xx - ux * xz, yz = ux * xy - uy * xx;
    const float hx = q2.x, hy = q2.y, hz = q2.z;
    const float bhx = uy * hz - uz * hy, bhy = uz * hx - ux * hz, bhz = ux * hy - uy * hx;
    const float ca = (hx * yx + hy * yy) + hz * yz;
    const float cb = (bhx * yx + bhy * yy) + bhz * yz;
    const float W = sqrtf(a_len * a_len * ca * ca + b_len * b_len * cb * cb);
    da = W > 0.0f ? k * a_len * ca * ca / W : 0.0f;
    db = W > 0.0f ? k * b_len * cb * cb / W : 0.0f;
}

constexpr int kMaxBwdSlices = 64;    // slices of one pixel deeper than a batch (more: HAIR_ERANGE)

template <int MODEL>
__global__ __launch_bounds__(kNT) void k_batch_bwd(FrameBufs f, ShadeArgs a, GradOut g, int S, int K) {
    __shared__ uint32_t s_cnt[kTilePix], s_kmin[kTilePix], s_kmax[kTilePix], s_off[kTilePix + 1];
    __shared__ uint32_t s_tmp[kNT];
    __shared__ __align__(16) uint2 s_B[kCap];
    __shared__ __align__(16) float s_work[4 * kCap];     // sort staging, then (alpha, L) -> adjoints
    __shared__ float s_T[kCap];                          // front-to-back transmittance before each fragment
    __shared__ float s_acc[6 * kNAcc];                   // per list entry partial sums
    __shared__ float s_dpix[4 * kTilePix];               // output adjoint of the batch's pixels
    __shared__ float s_agg[kNT * 4];
    __shared__ uint32_t s_aggh[kNT];
    // a pixel deeper than one batch: its slices (value range, by segment id inside key), their
    // composites (C rgb, T) and the boundary values each slice's adjoints need
    __shared__ unsigned long long s_range[2];
    __shared__ uint32_t s_slot, s_flag;
    __shared__ unsigned long long s_sl_lo[kMaxBwdSlices], s_sl_hi[kMaxBwdSlices];
    __shared__ uint32_t s_sl_key[kMaxBwdSlices], s_sl_n[kMaxBwdSlices];
    __shared__ float4 s_sl_agg[kMaxBwdSlices];
    __shared__ float4 s_sl_after[kMaxBwdSlices];        // (C rgb, S) of the slices behind
    __shared__ float s_sl_before[kMaxBwdSlices];         // T of the slices in front
    uint2* s_A = reinterpret_cast<uint2*>(s_work);
    uint32_t* s_bk = reinterpret_cast<uint32_t*>(s_work) + 2 * kCap;
    float4* s_p4 = reinterpret_cast<float4*>(s_work);

    const uint32_t n_batches = f.batch_start[f.T];
    const uint4 br = f.batches[blockIdx.x];
    if (blockIdx.x >= n_batches || f.ctr->cap_overflow) return;
    const BatchRec b = unpack_batch(br);
    const int tile = b.tile, p0 = b.p0, p1 = b.p1;
    const int t = threadIdx.x;
    const int px0 = (tile % f.ntx) * kTile, py0 = (tile / f.ntx) * kTile;
    const int W = a.cam.W, H = a.cam.H;
    const uint32_t lstart = f.tile_start[tile];
    const uint32_t n = f.tile_start[tile + 1] - lstart;
    const uint32_t* list = f.list + lstart;
    const size_t q = (size_t)tile * kTilePix + t;
    const uint32_t tile_off0 = f.pix_off[(size_t)tile * kTilePix + p0];
    if (t >= p0 && t < p1) {
        s_cnt[t] = f.pix_cnt[q];
        s_kmin[t] = f.pix_kmin[q];
        s_kmax[t] = f.pix_kmax[q];
        s_off[t] = f.pix_off[q] - tile_off0;
        const int gx = px0 + (t % kTile), gy = py0 + (t / kTile);
        const bool in = gx < W && gy < H;
        const float4 dp = in ? reinterpret_cast<const float4*>(g.d_rgba)[(size_t)gy * W + gx] : make_float4(0, 0, 0, 0);
        s_dpix[4 * t + 0] = dp.x; s_dpix[4 * t + 1] = dp.y; s_dpix[4 * t + 2] = dp.z; s_dpix[4 * t + 3] = dp.w;
    }
    if (t == 0) s_off[p1] = b.nfrag;
    for (int i = t; i < 6 * kNAcc; i += kNT) s_acc[i] = 0.0f;
    __syncthreads();
    const uint2* src = f.frags + b.frag0;

    // Steps 2-4 on the Fb records ordered in s_B (whole pixels, or one slice of one pixel).  A
    // slice's pixel starts with transmittance T_in (the slices in front) and ends over the
    // composite (C_out rgb, S_out) of the slices behind it; whole pixels start at 1 and end over
    // (0, 1).  grads = false: only the slice's own composite, into agg (C rgb, T).
    auto slice_core = [&](uint32_t Fb, float T_in, float4 out_c, bool grads, float4* agg) __attribute__((always_inline)) {
        // ---- 2. alpha and L per fragment (float)
        for (uint32_t i = t; i < Fb; i += kNT) {
            const uint2 rec = s_B[i];
            const uint32_t p = rec.y >> 24;
            const uint32_t gseg = list[rec.y & 0xFFFFFFu];
            float al, hh, L[3];
            shade_fragment<1, MODEL>(a, gseg, px0 + (int)(p % kTile), py0 + (int)(p / kTile), al, hh, L);
            s_p4[i] = make_float4(al, L[0], L[1], L[2]);
        }
        __syncthreads();
        // ---- 3a. forward: T before each fragment (segmented exclusive product over runs)
        const uint32_t run = (Fb + kNT - 1) / kNT;
        const uint32_t rb = min(Fb, t * run), re = min(Fb, rb + run);
        {
            float T = 1.f;
            uint32_t head = 0;
            for (uint32_t i = rb; i < re; ++i) {
                const uint32_t p = s_B[i].y >> 24;
                if (i == s_off[p]) { T = 1.f; head = 1; }
                T *= 1.0f - s_p4[i].x;
            }
            s_agg[4 * t + 3] = T;
            s_aggh[t] = head;
            __syncthreads();
            for (int off = 1; off < kNT; off <<= 1) {
                float tt = 1;
                uint32_t hh2 = 0;
                const bool has = t >= off;
                if (has) { tt = s_agg[4 * (t - off) + 3]; hh2 = s_aggh[t - off]; }
                __syncthreads();
                if (has && !s_aggh[t]) { s_agg[4 * t + 3] = tt * s_agg[4 * t + 3]; s_aggh[t] = hh2; }
                __syncthreads();
            }
            T = t > 0 ? s_agg[4 * (t - 1) + 3] : 1.f;
            for (uint32_t i = rb; i < re; ++i) {
                const uint32_t p = s_B[i].y >> 24;
                if (i == s_off[p]) T = 1.f;
                s_T[i] = T_in * T;
                T *= 1.0f - s_p4[i].x;
            }
            __syncthreads();
        }
        if (!grads) {   // the slice's own composite: C = sum T_k alpha_k L_k, T = prod (1 - alpha_k)
            float c0 = 0.f, c1 = 0.f, c2 = 0.f;
            for (uint32_t i = t; i < Fb; i += kNT) {
                const float4 v = s_p4[i];
                const float w = s_T[i] * v.x;
                c0 += w * v.y;
                c1 += w * v.z;
                c2 += w * v.w;
            }
            s_agg[4 * t + 0] = c0; s_agg[4 * t + 1] = c1; s_agg[4 * t + 2] = c2;
            __syncthreads();
            if (t == 0) {
                float4 r = make_float4(0.f, 0.f, 0.f, 1.f);
                for (int i = 0; i < kNT; ++i) { r.x += s_agg[4 * i]; r.y += s_agg[4 * i + 1]; r.z += s_agg[4 * i + 2]; }
                if (Fb) r.w = s_T[Fb - 1] * (1.0f - s_p4[Fb - 1].x);
                *agg = r;
            }
            __syncthreads();
            return;
        }
        // ---- 3b. backward: suffix composite (C+, S+) after each fragment, then the adjoints
        {
            // run aggregate from the run start through its first pixel end (or the whole run)
            float C0 = 0.f, C1 = 0.f, C2 = 0.f, Sx = 1.f;
            uint32_t tail = 0;
            for (uint32_t i = re; i > rb; --i) {
                const uint32_t k = i - 1;
                const uint32_t p = s_B[k].y >> 24;
                if (k + 1 == s_off[p] + s_cnt[p]) { C0 = C1 = C2 = 0.f; Sx = 1.f; tail = 1; }
                const float4 v = s_p4[k];
                C0 = v.x * v.y + (1.0f - v.x) * C0;
                C1 = v.x * v.z + (1.0f - v.x) * C1;
                C2 = v.x * v.w + (1.0f - v.x) * C2;
                Sx = (1.0f - v.x) * Sx;
            }
            s_agg[4 * t + 0] = C0; s_agg[4 * t + 1] = C1; s_agg[4 * t + 2] = C2; s_agg[4 * t + 3] = Sx;
            s_aggh[t] = tail;
            __syncthreads();
            // right-to-left inclusive scan: R_t = agg_t.tail ? agg_t : agg_t over R_{t+1}
            for (int off = 1; off < kNT; off <<= 1) {
                float c0 = 0, c1 = 0, c2 = 0, ss = 1;
                const bool has = t + off < kNT;
                if (has) {
                    c0 = s_agg[4 * (t + off) + 0]; c1 = s_agg[4 * (t + off) + 1];
                    c2 = s_agg[4 * (t + off) + 2]; ss = s_agg[4 * (t + off) + 3];
                }
                const uint32_t my_tail = s_aggh[t];
                const uint32_t r_tail = has ? s_aggh[t + off] : 0u;
                __syncthreads();
                if (has && !my_tail) {
                    const float mS = s_agg[4 * t + 3];
                    s_agg[4 * t + 0] = s_agg[4 * t + 0] + mS * c0;
                    s_agg[4 * t + 1] = s_agg[4 * t + 1] + mS * c1;
                    s_agg[4 * t + 2] = s_agg[4 * t + 2] + mS * c2;
                    s_agg[4 * t + 3] = mS * ss;
                    s_aggh[t] = r_tail;
                }
                __syncthreads();
            }
            if (t + 1 < kNT) { C0 = s_agg[4 * (t + 1) + 0]; C1 = s_agg[4 * (t + 1) + 1]; C2 = s_agg[4 * (t + 1) + 2]; Sx = s_agg[4 * (t + 1) + 3]; }
            else { C0 = C1 = C2 = 0.f; Sx = 1.f; }
            __syncthreads();
            for (uint32_t i = re; i > rb; --i) {
                const uint32_t k = i - 1;
                const uint32_t p = s_B[k].y >> 24;
                if (k + 1 == s_off[p] + s_cnt[p]) { C0 = C1 = C2 = 0.f; Sx = 1.f; }
                const float4 v = s_p4[k];
                const float Tk = s_T[k];
                const float dR = s_dpix[4 * p + 0], dG = s_dpix[4 * p + 1], dB = s_dpix[4 * p + 2], dA = s_dpix[4 * p + 3];
                // behind fragment k: the rest of its pixel's records here, then what lies behind
                const float Ca0 = C0 + Sx * out_c.x, Ca1 = C1 + Sx * out_c.y, Ca2 = C2 + Sx * out_c.z;
                const float Sa = Sx * out_c.w;
                const float g_alpha = Tk * (dR * (v.y - Ca0) + dG * (v.z - Ca1) + dB * (v.w - Ca2) + dA * Sa);
                const float ta = Tk * v.x;
                C0 = v.x * v.y + (1.0f - v.x) * C0;
                C1 = v.x * v.z + (1.0f - v.x) * C1;
                C2 = v.x * v.w + (1.0f - v.x) * C2;
                Sx = (1.0f - v.x) * Sx;
                s_p4[k] = make_float4(g_alpha, dR * ta, dG * ta, dB * ta);
            }
        }
        __syncthreads();
        // ---- 4. partials: alpha and L as Dual6, contracted with the adjoints.  A fragment whose
        // four adjoints are all zero (behind an opaque fragment of its pixel, T_k = 0, or in a
        // pixel without output adjoint) contributes exactly nothing; the others are listed first
        // (in s_T, free after step 3) so that every lane's Dual6 work is a fragment that counts.
        uint32_t* s_idx = reinterpret_cast<uint32_t*>(s_T);
        uint32_t n_live;
        {
            uint32_t mine = 0;
            for (uint32_t i = t; i < Fb; i += kNT) {
                const float4 v = s_p4[i];
                mine += (v.x != 0.0f || v.y != 0.0f || v.z != 0.0f || v.w != 0.0f) ? 1u : 0u;
            }
            uint32_t pos;
            n_live = block_exscan_u32(mine, s_tmp, pos);
            for (uint32_t i = t; i < Fb; i += kNT) {
                const float4 v = s_p4[i];
                if (v.x != 0.0f || v.y != 0.0f || v.z != 0.0f || v.w != 0.0f) s_idx[pos++] = i;
            }
            __syncthreads();
        }
        for (uint32_t kk = t; kk < n_live; kk += kNT) {
            const uint32_t i = s_idx[kk];
            const uint2 rec = s_B[i];
            const uint32_t p = rec.y >> 24;
            const uint32_t j = rec.y & 0xFFFFFFu;
            const uint32_t gseg = list[j];
            const float4 adj = s_p4[i];
            const SegRec s = a.seg[gseg];
            const ShadeRec& srec = a.shade[gseg];
            const float4 q0 = srec.q0, q1 = srec.q1, q2 = srec.q2, q3 = srec.q3;
            float dha, dhb;
            halfwidth_partials(a.cam, s, q0, q1, q2, q3.x, q3.y, dha, dhb);
            Dual6 hw(s.hw);
            hw.d[0] = dha;
            hw.d[1] = dhb;
            const Dual6 al = Dual6::seed(q3.x, 0), bl = Dual6::seed(q3.y, 1), rr = Dual6::seed(q3.w, 2);
            const Dual6 sig[3] = {Dual6::seed(q0.w, 3), Dual6::seed(q1.w, 4), Dual6::seed(q2.w, 5)};
            Dual6 alpha, hoff, L[3];
            shade_core<1, MODEL, Dual6>(a, s, q0, q1, q2, q3.z, px0 + (int)(p % kTile), py0 + (int)(p / kTile), hw, al,
                                        bl, rr, sig, alpha, hoff, L);
            float gp[6];
#pragma unroll
            for (int m = 0; m < 6; ++m)
                gp[m] = adj.x * alpha.d[m] + adj.y * L[0].d[m] + adj.z * L[1].d[m] + adj.w * L[2].d[m];
            if (j < (uint32_t)kNAcc) {
#pragma unroll
                for (int m = 0; m < 6; ++m) atomicAdd(&s_acc[m * kNAcc + j], gp[m]);
            } else {
                const uint32_t par = g.rows ? g.rows[gseg] >> 6 : gseg;   // a piece's segment
                const int owner = (int)par / S;
                atomicAdd(&g.d_axes[2 * par], gp[0]);
                atomicAdd(&g.d_axes[2 * par + 1], gp[1]);
                atomicAdd(&g.d_r[owner], gp[2]);
                atomicAdd(&g.d_sig[owner], gp[3]);
                atomicAdd(&g.d_sig[K + owner], gp[4]);
                atomicAdd(&g.d_sig[2 * K + owner], gp[5]);
            }
        }
        __syncthreads();
    };

    if (!b.over) {
        const uint32_t Fb = b.nfrag;
        for (uint32_t i = t; i < Fb; i += kNT) {
            s_A[i] = src[i];
            s_bk[i] = 0;
        }
        __syncthreads();
        order_batch_insertion(Fb, s_cnt, s_kmin, s_kmax, s_off, s_tmp, s_A, s_B, s_bk, list);
        slice_core(Fb, 1.0f, make_float4(0.f, 0.f, 0.f, 1.f), true, nullptr);
    } else {
        // ---- a pixel deeper than one batch: the forward's slices in (key, segment id) order,
        // each differentiated with the transmittance of the slices in front of it and the
        // composite of the slices behind it (two sweeps: composites, then adjoints)
        const int p = p0;
        const uint32_t k = b.nfrag;
        const unsigned long long key_end = (unsigned long long)s_kmax[p] + 1ull;
        auto by_key = [&](const uint2& r, uint32_t& v) { v = r.x; return true; };
        // stage the records of slice [v_lo, v_hi) (by key, or inside key K0 by segment id) in
        // s_B, ordered, as a one-pixel batch
        auto stage = [&](uint32_t Fb, unsigned long long v_lo, unsigned long long v_hi, bool by_seg, uint32_t K0)
            __attribute__((always_inline)) {
            if (t == 0) s_slot = 0;
            __syncthreads();
            for (uint32_t i = t; i < k; i += kNT) {
                const uint2 r = src[i];
                uint32_t v = r.x;
                bool in = true;
                if (by_seg) {
                    in = r.x == K0;
                    if (in) v = list[r.y & 0xFFFFFFu];
                }
                if (in && (unsigned long long)v >= v_lo && (unsigned long long)v < v_hi)
                    s_A[atomicAdd(&s_slot, 1u)] = make_uint2(v, r.y);
            }
            __syncthreads();
            for (uint32_t i = t; i < Fb; i += kNT) s_bk[i] = 0;
            if (t == 0) {
                s_cnt[p] = Fb;
                s_kmin[p] = (uint32_t)v_lo;
                s_kmax[p] = (uint32_t)(v_hi - 1);
                s_off[p] = 0;
                s_off[p + 1] = Fb;
            }
            __syncthreads();
            order_batch_insertion(Fb, s_cnt, s_kmin, s_kmax, s_off, s_tmp, s_A, s_B, s_bk, list);
        };
        uint32_t nsl = 0;
        bool ok = true;
        auto add_slice = [&](uint32_t Fb, unsigned long long v_lo, unsigned long long v_hi, bool by_seg, uint32_t K0)
            __attribute__((always_inline)) {
            if (nsl >= (uint32_t)kMaxBwdSlices) { ok = false; return; }
            stage(Fb, v_lo, v_hi, by_seg, K0);
            slice_core(Fb, 1.0f, make_float4(0.f, 0.f, 0.f, 1.f), false, &s_sl_agg[nsl]);
            if (t == 0) {
                s_sl_lo[nsl] = v_lo;
                s_sl_hi[nsl] = v_hi;
                s_sl_key[nsl] = by_seg ? K0 : 0xFFFFFFFFu;
                s_sl_n[nsl] = Fb | (by_seg ? 0x80000000u : 0u);
            }
            ++nsl;
        };
        unsigned long long lo = s_kmin[p];
        while (ok && lo < key_end) {
            unsigned long long hi;
            uint32_t Fb;
            const uint32_t flag = refine_slice(k, src, lo, key_end, by_key, s_bk, s_tmp, s_range, s_slot, s_flag, hi, Fb);
            if (flag == 0) {
                if (Fb) add_slice(Fb, lo, hi, false, 0u);
                lo = hi;
                continue;
            }
            const uint32_t K0 = (uint32_t)lo;
            auto by_seg = [&](const uint2& r, uint32_t& v) {
                if (r.x != K0) return false;
                v = list[r.y & 0xFFFFFFu];
                return true;
            };
            unsigned long long slo = 0;
            const unsigned long long send = 1ull << 32;
            while (ok && slo < send) {
                unsigned long long shi;
                if (refine_slice(k, src, slo, send, by_seg, s_bk, s_tmp, s_range, s_slot, s_flag, shi, Fb) != 0) {
                    ok = false;
                    break;
                }
                if (Fb) add_slice(Fb, slo, shi, true, K0);
                slo = shi;
            }
            lo = (unsigned long long)K0 + 1ull;
        }
        if (!ok) {   // more slices than the kernel keeps: reported, not differentiated
            if (t == 0) atomicAdd(&f.ctr->overflow_pixels, 1u);
            return;
        }
        if (t == 0) {   // transmittance in front of each slice and the composite behind it
            float T = 1.f;
            for (uint32_t i = 0; i < nsl; ++i) {
                s_sl_before[i] = T;
                T *= s_sl_agg[i].w;
            }
            float4 behind = make_float4(0.f, 0.f, 0.f, 1.f);
            for (uint32_t i = nsl; i > 0; --i) {
                s_sl_after[i - 1] = behind;
                const float4 c = s_sl_agg[i - 1];
                behind = make_float4(c.x + c.w * behind.x, c.y + c.w * behind.y, c.z + c.w * behind.z, c.w * behind.w);
            }
        }
        __syncthreads();
        for (uint32_t i = 0; i < nsl; ++i) {
            const uint32_t Fb = s_sl_n[i] & 0x7FFFFFFFu;
            const bool by_seg = (s_sl_n[i] >> 31) != 0;
            stage(Fb, s_sl_lo[i], s_sl_hi[i], by_seg, s_sl_key[i]);
            slice_core(Fb, s_sl_before[i], s_sl_after[i], true, nullptr);
        }
    }
    const uint32_t nacc = min(n, (uint32_t)kNAcc);
    for (uint32_t j = t; j < nacc; j += kNT) {
        float v[6];
        bool any = false;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            v[m] = s_acc[m * kNAcc + j];
            any |= v[m] != 0.0f;
        }
        if (!any) continue;
        const uint32_t gseg = list[j];
        const uint32_t par = g.rows ? g.rows[gseg] >> 6 : gseg;
        const int owner = (int)par / S;
        atomicAdd(&g.d_axes[2 * par], v[0]);
        atomicAdd(&g.d_axes[2 * par + 1], v[1]);
        atomicAdd(&g.d_r[owner], v[2]);
        atomicAdd(&g.d_sig[owner], v[3]);
        atomicAdd(&g.d_sig[K + owner], v[4]);
        atomicAdd(&g.d_sig[2 * K + owner], v[5]);
    }
}

// ---------------------------------------------------------------------------------------
// Thick-hair construction (Sec. 5.1 step 3), float64 sums in member order.
__global__ void k_build_centers(const float* __restrict__ vx, const float* __restrict__ vy,
                                const float* __restrict__ vz, const float* __restrict__ width,
                                const float* __restrict__ sig, int n_strands, int V,
                                const int32_t* __restrict__ members, const int32_t* __restrict__ mstart, int K,
                                float* cx, float* cy, float* cz, float* r, float* csig, int32_t* n_total) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= K * V) return;
    const int c = g / V, k = g - c * V;
    const int b = mstart[c], e = mstart[c + 1];
    double sx = 0, sy = 0, sz = 0;
    for (int m = b; m < e; ++m) {
        const int v = members[m] * V + k;
        sx += (double)vx[v];
        sy += (double)vy[v];
        sz += (double)vz[v];
    }
    const double N = (double)(e - b);
    cx[g] = (float)(sx / N);
    cy[g] = (float)(sy / N);
    cz[g] = (float)(sz / N);
    if (k == 0) {
        double sw = 0, s0 = 0, s1 = 0, s2 = 0;
        for (int m = b; m < e; ++m) {
            const int s = members[m];
            sw += (double)width[s];
            s0 += (double)sig[s];
            s1 += (double)sig[n_strands + s];
            s2 += (double)sig[2 * n_strands + s];
        }
        r[c] = (float)((sw / N) * 0.5);
        csig[c] = (float)(s0 / N);
        csig[K + c] = (float)(s1 / N);
        csig[2 * K + c] = (float)(s2 / N);
        n_total[c] = e - b;
    }
}

__global__ void k_build_ellipses(const float* __restrict__ vx, const float* __restrict__ vy,
                                 const float* __restrict__ vz, int V, const int32_t* __restrict__ members,
                                 const int32_t* __restrict__ mstart, int K, const float* __restrict__ cx,
                                 const float* __restrict__ cy, const float* __restrict__ cz,
                                 const float* __restrict__ r, float* ahat, float* axes) {
    const int S = V - 1;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= K * S) return;
    const int c = g / S, k = g - c * S;
    const int ia = c * V + k;
    const double ax = cx[ia], ay = cy[ia], az = cz[ia];
    const double bx = cx[ia + 1], by = cy[ia + 1], bz = cz[ia + 1];
    double ux = bx - ax, uy = by - ay, uz = bz - az;
    const double ul = sqrt(ux * ux + uy * uy + uz * uz);
    ux /= ul; uy /= ul; uz /= ul;
    // basis of the plane orthogonal to u: start from the axis of smallest |u_j| (lowest index on ties)
    const double fx = fabs(ux), fy = fabs(uy), fz = fabs(uz);
    int j = 0;
    if (fy < fx) j = 1;
    if (fz < (j == 0 ? fx : fy)) j = 2;
    double ex = j == 0, ey = j == 1, ez = j == 2;
    const double eu = ex * ux + ey * uy + ez * uz;
    ex -= eu * ux; ey -= eu * uy; ez -= eu * uz;
    const double el = sqrt(ex * ex + ey * ey + ez * ez);
    ex /= el; ey /= el; ez /= el;
    const double fx2 = uy * ez - uz * ey, fy2 = uz * ex - ux * ez, fz2 = ux * ey - uy * ex;
    const double mx = 0.5 * (ax + bx), my = 0.5 * (ay + by), mz = 0.5 * (az + bz);
    const int b0 = mstart[c], b1 = mstart[c + 1];
    double c11 = 0, c12 = 0, c22 = 0;
    for (int m = b0; m < b1; ++m) {
        const int v = members[m] * V + k;
        const double qx = 0.5 * ((double)vx[v] + (double)vx[v + 1]) - mx;
        const double qy = 0.5 * ((double)vy[v] + (double)vy[v + 1]) - my;
        const double qz = 0.5 * ((double)vz[v] + (double)vz[v + 1]) - mz;
        const double q1 = qx * ex + qy * ey + qz * ez;
        const double q2 = qx * fx2 + qy * fy2 + qz * fz2;
        c11 += q1 * q1;
        c12 += q1 * q2;
        c22 += q2 * q2;
    }
    const double N = (double)(b1 - b0);
    c11 /= N; c12 /= N; c22 /= N;
    const double hm = 0.5 * (c11 + c22), hd = 0.5 * (c11 - c22);
    const double rad = sqrt(hd * hd + c12 * c12);
    const double l1 = fmax(hm + rad, 0.0), l2 = fmax(hm - rad, 0.0);
    double v1 = 1.0, v2 = 0.0;
    if (!((l1 - l2) <= 1e-12 * (l1 + l2))) {
        // eigenvector of l1: (l1 - c22, c12) or (c12, l1 - c11), the better conditioned
        const double a1 = l1 - c22, a2 = c12, b1v = c12, b2 = l1 - c11;
        if (a1 * a1 + a2 * a2 >= b1v * b1v + b2 * b2) { v1 = a1; v2 = a2; } else { v1 = b1v; v2 = b2; }
        const double vl = sqrt(v1 * v1 + v2 * v2);
        v1 /= vl; v2 /= vl;
    }
    const int nseg = K * S;
    ahat[g] = (float)(v1 * ex + v2 * fx2);
    ahat[nseg + g] = (float)(v1 * ey + v2 * fy2);
    ahat[2 * nseg + g] = (float)(v1 * ez + v2 * fz2);
    const double rr = (double)r[c];
    axes[2 * g] = (float)(rr + 2.0 * sqrt(l1));
    axes[2 * g + 1] = (float)(rr + 2.0 * sqrt(l2));
}

inline int blocks_for(size_t n, int per) { return (int)((n + per - 1) / per); }


// ---------------------------------------------------------------------------------------
// Curved thick hairs: the centre line is the uniform Catmull-Rom spline through the level's
// centre vertices (ends clamped), each segment split into m equal parameter steps by its
// screen length (Sec. 5.2, tessellation by distance; Sec. 6, spline centre lines).  The
// points decide integers (snapped endpoints), so the basis is evaluated with one rounding
// per operation in a fixed order; u = 0 and u = 1 return the vertices themselves.

__device__ inline void spline_point(const LevelDev& lv, int owner, int k, float u, float& x, float& y, float& z) {
    const int base = owner * (lv.S + 1);
    if (u == 0.0f || u == 1.0f) {
        const int i = base + k + (u == 1.0f ? 1 : 0);
        x = lv.vx[i];
        y = lv.vy[i];
        z = lv.vz[i];
        return;
    }
    const int i0 = base + max(k - 1, 0), i1 = base + k, i2 = base + k + 1, i3 = base + min(k + 2, lv.S);
    const float u2 = u * u, u3 = u2 * u;
    const float w0 = 0.5f * ((2.0f * u2 - u3) - u);
    const float w1 = 0.5f * ((3.0f * u3 - 5.0f * u2) + 2.0f);
    const float w2 = 0.5f * ((4.0f * u2 - 3.0f * u3) + u);
    const float w3 = 0.5f * (u3 - u2);
    x = ((w0 * lv.vx[i0] + w1 * lv.vx[i1]) + w2 * lv.vx[i2]) + w3 * lv.vx[i3];
    y = ((w0 * lv.vy[i0] + w1 * lv.vy[i1]) + w2 * lv.vy[i2]) + w3 * lv.vy[i3];
    z = ((w0 * lv.vz[i0] + w1 * lv.vz[i1]) + w2 * lv.vz[i2]) + w3 * lv.vz[i3];
}

// Steps of segment g: the smallest m in [1, max_sub] with (m T16)^2 >= dX^2 + dY^2 (snapped
// screen extent of the straight segment); 1 when an endpoint is not on screen.
__global__ __launch_bounds__(256) void k_tess_count(LevelDev lv, CamConst cam, int T16, int max_sub,
                                                    uint32_t* __restrict__ cnt) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= lv.nseg) return;
    const int owner = g / lv.S, k = g - owner * lv.S;
    const int va = owner * (lv.S + 1) + k;
    const PPoint A = project_point(cam, lv.vx[va], lv.vy[va], lv.vz[va]);
    const PPoint B = project_point(cam, lv.vx[va + 1], lv.vy[va + 1], lv.vz[va + 1]);
    int m = 1;
    if (A.ok && B.ok) {
        const long long dx = (long long)rintf(B.X16) - (long long)rintf(A.X16);
        const long long dy = (long long)rintf(B.Y16) - (long long)rintf(A.Y16);
        const long long d2 = dx * dx + dy * dy;
        while (m < max_sub && (long long)(m * T16) * (long long)(m * T16) < d2) ++m;
    }
    cnt[g] = (uint32_t)m;
}

// Row list: g << 4 | j for the m steps j of every segment g, at start[g].
__global__ __launch_bounds__(256) void k_tess_fill(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ start,
                                                   int nseg, uint32_t* __restrict__ rows) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nseg) return;
    const uint32_t m = cnt[g], o = start[g];
    for (uint32_t j = 0; j < m; ++j) rows[o + j] = ((uint32_t)g << 4) | j;
}

// Row r: step j of segment g, from P(j / m) to P((j + 1) / m), with segment g's cross-section.
__global__ __launch_bounds__(256) void k_project_tess(LevelDev lv, const uint32_t* __restrict__ rows, int nrows,
                                                      const uint32_t* __restrict__ cnt, CamConst cam,
                                                      SegRec* __restrict__ seg, ShadeRec* __restrict__ shade) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const uint32_t e = rows[r];
    const int g = (int)(e >> 4), j = (int)(e & 15u);
    const int m = (int)cnt[g];
    const int owner = g / lv.S, k = g - owner * lv.S;
    float ax, ay, az, bx, by, bz;
    spline_point(lv, owner, k, (float)j / (float)m, ax, ay, az);
    spline_point(lv, owner, k, (float)(j + 1) / (float)m, bx, by, bz);
    seg[r] = project_segment_at(lv, g, ax, ay, az, bx, by, bz, cam, shade + r);
}

// ---------------------------------------------------------------------------------------
// Long segments (an axis extent above kMaxAxis sub-pixels, both endpoints on the guard band)
// are drawn as m = min(ceil(extent / kSplitLen), kMaxPieces) pieces of equal screen parameter:
// piece j runs between the world points of screen parameters j / m and (j + 1) / m, found
// with the perspective-correct parameter t_w = s izB / (izA + s (izB - izA)) in float32 (one
// rounding per operation) and exact at s = 0 and 1.  A piece keeps its segment's attributes.
__device__ inline uint32_t split_pieces(const LevelDev& lv, int g, const CamConst& cam) {
    const int owner = g / lv.S, k = g - owner * lv.S;
    const int va = owner * (lv.S + 1) + k;
    const PPoint A = project_point(cam, lv.vx[va], lv.vy[va], lv.vz[va]);
    const PPoint B = project_point(cam, lv.vx[va + 1], lv.vy[va + 1], lv.vz[va + 1]);
    int m = 1;
    if (A.ok && B.ok) {
        const int dx = abs((int)rintf(B.X16) - (int)rintf(A.X16)), dy = abs((int)rintf(B.Y16) - (int)rintf(A.Y16));
        const int ext = max(dx, dy);
        if (ext > kMaxAxis) m = min((ext + kSplitLen - 1) / kSplitLen, kMaxPieces);
    }
    return (uint32_t)m;
}

__global__ __launch_bounds__(256) void k_split_count(LevelDev lv, CamConst cam, uint32_t* __restrict__ cnt) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= lv.nseg) return;
    cnt[g] = split_pieces(lv, g, cam);
}

// The same over the rows of a mixed frame (sel[i] = level << 28 | segment of that level).
__global__ __launch_bounds__(256) void k_split_count_mixed(HierDev h, const uint32_t* __restrict__ sel, int nsel,
                                                           CamConst cam, uint32_t* __restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsel) return;
    const uint32_t e = sel[i];
    cnt[i] = split_pieces(h.lv[e >> 28], (int)(e & 0x0FFFFFFFu), cam);
}

// Row list: g << 6 | j for the m pieces j of every segment g, at start[g].
__global__ __launch_bounds__(256) void k_split_fill(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ start,
                                                    int nseg, uint32_t* __restrict__ rows) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nseg) return;
    const uint32_t m = cnt[g], o = start[g];
    for (uint32_t j = 0; j < m; ++j) rows[o + j] = ((uint32_t)g << 6) | j;
}

__device__ inline void split_point(float ax, float ay, float az, float bx, float by, float bz, float izA, float izB,
                                   int j, int m, float& x, float& y, float& z) {
    if (j == 0) { x = ax; y = ay; z = az; return; }
    if (j == m) { x = bx; y = by; z = bz; return; }
    const float s = (float)j / (float)m;
    const float iz = izA + s * (izB - izA);
    const float tw = (s * izB) / iz;
    x = ax + tw * (bx - ax);
    y = ay + tw * (by - ay);
    z = az + tw * (bz - az);
}

// Piece j of m of segment g of lv (the whole segment when m = 1).
__device__ inline SegRec project_piece(const LevelDev& lv, int g, int j, int m, const CamConst& cam, ShadeRec* sr,
                                       bool packed) {
    if (m == 1) return project_segment(lv, g, cam, sr, packed);
    const int owner = g / lv.S, k = g - owner * lv.S;
    const int va = owner * (lv.S + 1) + k;
    const float ax = lv.vx[va], ay = lv.vy[va], az = lv.vz[va];
    const float bx = lv.vx[va + 1], by = lv.vy[va + 1], bz = lv.vz[va + 1];
    const PPoint A = project_point(cam, ax, ay, az), B = project_point(cam, bx, by, bz);
    float p0x, p0y, p0z, p1x, p1y, p1z;
    split_point(ax, ay, az, bx, by, bz, A.iz, B.iz, j, m, p0x, p0y, p0z);
    split_point(ax, ay, az, bx, by, bz, A.iz, B.iz, j + 1, m, p1x, p1y, p1z);
    return project_segment_at(lv, g, p0x, p0y, p0z, p1x, p1y, p1z, cam, sr, packed);
}

// Row r: piece j of segment g (a whole segment when it has one piece), with segment g's
// attributes; strand levels write the packed strand shading record.
__global__ __launch_bounds__(256) void k_project_split(LevelDev lv, const uint32_t* __restrict__ rows, int nrows,
                                                       const uint32_t* __restrict__ cnt, CamConst cam,
                                                       SegRec* __restrict__ seg, ShadeRec* __restrict__ shade) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const uint32_t e = rows[r];
    const int g = (int)(e >> 6), j = (int)(e & 63u);
    ShadeRec sr;
    sr.q3 = make_float4(0.f, 0.f, 0.f, 0.f);
    seg[r] = project_piece(lv, g, j, (int)cnt[g], cam, &sr, lv.kind == 0);
    shade[r] = sr;
}

// Row r of a mixed frame drawn in pieces: piece j of selection row i (rows[r] = i << 6 | j),
// with the record layout of k_project_mixed.
__global__ __launch_bounds__(256) void k_project_split_mixed(HierDev h, const uint32_t* __restrict__ sel,
                                                             const uint32_t* __restrict__ rows, int nrows,
                                                             const uint32_t* __restrict__ cnt, CamConst cam,
                                                             SegRec* __restrict__ seg, ShadeRec* __restrict__ shade) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const uint32_t e = rows[r];
    const int i = (int)(e >> 6), j = (int)(e & 63u);
    const uint32_t s = sel[i];
    const int L = (int)(s >> 28), g = (int)(s & 0x0FFFFFFFu);
    SegRec rec = project_piece(h.lv[L], g, j, (int)cnt[i], cam, shade + r, false);
    if (h.lv[L].kind == 1) rec.hwfx |= kFlagThick;
    else shade[r].q3 = make_float4(0.5f * h.lv[L].width[g / h.lv[L].S], 0.0f, 0.0f, -1.0f);
    seg[r] = rec;
}

// ---------------------------------------------------------------------------------------
// Shadow pass: deep opacity map toward a directional light (Sec. 5.2 shadow pass; its count
// feeds the forward lobes of Sec. 4).  The light view is an orthographic raster with the
// camera pass's integer coverage rule, so binning, counting and emission are the camera
// kernels; only the projection and the per-texel resolve are the light's own.  Every float
// step that decides an integer (bounds, grid, snapping, depth) is a single rounding per
// operation in a fixed order (this file is compiled without contraction).


// World half-width padding the grid: a strand's radius, a thick hair's larger semi-axis.
__device__ inline float pad_halfwidth(const LevelDev& lv, int g) {
    return lv.kind == 0 ? 0.5f * lv.width[g / lv.S] : fmaxf(lv.axes[2 * g], lv.axes[2 * g + 1]);
}

// A mixed frame's shadow pass reads its rows from the camera pass's shading records instead
// of a level: q0.xyz, q1.xyz the world endpoints, q2.xyz a^, and q3 = (|a|, |b|, n_total, r)
// for a thick hair or (radius, 0, 0, -1) for a strand.
__device__ inline bool row_is_strand(const ShadeRec& r) { return r.q3.w < 0.0f; }

// Endpoints of segment (or row) g.
__device__ inline void dom_endpoints(const LevelDev& lv, const ShadeRec* rows, int g, float& ax, float& ay, float& az,
                                     float& bx, float& by, float& bz) {
    if (rows) {
        const float4 q0 = rows[g].q0, q1 = rows[g].q1;
        ax = q0.x; ay = q0.y; az = q0.z;
        bx = q1.x; by = q1.y; bz = q1.z;
        return;
    }
    const int owner = g / lv.S, k = g - owner * lv.S;
    const int va = owner * (lv.S + 1) + k;
    ax = lv.vx[va]; ay = lv.vy[va]; az = lv.vz[va];
    bx = lv.vx[va + 1]; by = lv.vy[va + 1]; bz = lv.vz[va + 1];
}

constexpr int kDomBoundThreads = 256;
constexpr int kDomBoundMaxBlocks = 1024;

// Per block: (min u - w, max u + w, min v - w, max v + w, max z) over its segments' endpoints.
__global__ __launch_bounds__(kDomBoundThreads) void k_dom_bounds(LevelDev lv, const ShadeRec* __restrict__ rows,
                                                                DomBasis b, float* __restrict__ part) {
    __shared__ float s_red[5][kDomBoundThreads];
    float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, zmax = -INFINITY;
    for (int g = blockIdx.x * kDomBoundThreads + threadIdx.x; g < lv.nseg; g += gridDim.x * kDomBoundThreads) {
        float pe[2][3];
        dom_endpoints(lv, rows, g, pe[0][0], pe[0][1], pe[0][2], pe[1][0], pe[1][1], pe[1][2]);
        const float w = !rows ? pad_halfwidth(lv, g)
                              : (row_is_strand(rows[g]) ? rows[g].q3.x : fmaxf(rows[g].q3.x, rows[g].q3.y));
        for (int e = 0; e < 2; ++e) {
            const float x = pe[e][0], y = pe[e][1], z = pe[e][2];
            const float u = dot_e(b.e1, x, y, z), v = dot_e(b.e2, x, y, z), d = dot_e(b.d, x, y, z);
            umin = fminf(umin, u - w);
            umax = fmaxf(umax, u + w);
            vmin = fminf(vmin, v - w);
            vmax = fmaxf(vmax, v + w);
            zmax = fmaxf(zmax, d);
        }
    }
    const int t = threadIdx.x;
    s_red[0][t] = umin; s_red[1][t] = -umax; s_red[2][t] = vmin; s_red[3][t] = -vmax; s_red[4][t] = -zmax;
    __syncthreads();
    for (int h = kDomBoundThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int c = 0; c < 5; ++c) s_red[c][t] = fminf(s_red[c][t], s_red[c][t + h]);
        __syncthreads();
    }
    if (t < 5) part[5 * blockIdx.x + t] = s_red[t][0];
}

// One block: reduce the partial bounds and set the grid (texel size = extent / (R - 2), one
// texel of margin; z_ref = z_max + 1 so that iz = z_ref - z >= 1 orders like inverse depth).
__global__ __launch_bounds__(kDomBoundThreads) void k_dom_grid(const float* __restrict__ part, int nb, DomBasis b,
                                                             int R, DomGrid* __restrict__ grid) {
    __shared__ float s_red[5][kDomBoundThreads];
    const int t = threadIdx.x;
    float m[5] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
    for (int i = t; i < nb; i += kDomBoundThreads)
        for (int c = 0; c < 5; ++c) m[c] = fminf(m[c], part[5 * i + c]);
    for (int c = 0; c < 5; ++c) s_red[c][t] = m[c];
    __syncthreads();
    for (int h = kDomBoundThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int c = 0; c < 5; ++c) s_red[c][t] = fminf(s_red[c][t], s_red[c][t + h]);
        __syncthreads();
    }
    if (t == 0) {
        const float umin = s_red[0][0], umax = -s_red[1][0], vmin = s_red[2][0], vmax = -s_red[3][0];
        const float zmax = -s_red[4][0];
        const float ext = fmaxf(fmaxf(umax - umin, vmax - vmin), 1e-6f);
        DomGrid gr;
        gr.b = b;
        gr.s = ext / (float)(R - 2);
        gr.u0 = umin - gr.s;
        gr.v0 = vmin - gr.s;
        gr.k16 = 16.0f / gr.s;
        gr.z_ref = zmax + 1.0f;
        gr.R = R;
        *grid = gr;
    }
}

// Light-view record of segment g: snapped texel coordinates (1/16 texel), iz = z_ref - z, and
// the half-width in texels (a strand's radius; a thick hair's support across the light).
__global__ __launch_bounds__(256) void k_project_light(LevelDev lv, const ShadeRec* __restrict__ rows,
                                                       const DomGrid* __restrict__ grid, SegRec* __restrict__ seg) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= lv.nseg) return;
    const DomGrid gr = *grid;
    const int owner = g / lv.S;
    float ax, ay, az, bx, by, bz;
    dom_endpoints(lv, rows, g, ax, ay, az, bx, by, bz);
    const bool strand = rows ? row_is_strand(rows[g]) : lv.kind == 0;
    float hw;
    if (strand) {
        hw = (rows ? rows[g].q3.x : 0.5f * lv.width[owner]) / gr.s;
    } else {
        const float tx = bx - ax, ty = by - ay, tz = bz - az;
        const float tl = norm3f(tx, ty, tz);
        const float ux = tx / tl, uy = ty / tl, uz = tz / tl;
        const float wx = gr.b.omega[0], wy = gr.b.omega[1], wz = gr.b.omega[2];
        const float dwu = (wx * ux + wy * uy) + wz * uz;
        const float px = wx - dwu * ux, py = wy - dwu * uy, pz = wz - dwu * uz;
        const float pl = norm3f(px, py, pz);
        const float xx = px / pl, xy = py / pl, xz = pz / pl;
        const float yx = uy * xz - uz * xy, yy = uz * xx - ux * xz, yz = ux * xy - uy * xx;
        const float hx = rows ? rows[g].q2.x : lv.ahat[g];
        const float hy = rows ? rows[g].q2.y : lv.ahat[lv.nseg + g];
        const float hz = rows ? rows[g].q2.z : lv.ahat[2 * lv.nseg + g];
        const float bhx = uy * hz - uz * hy, bhy = uz * hx - ux * hz, bhz = ux * hy - uy * hx;
        const float a_len = rows ? rows[g].q3.x : lv.axes[2 * g], b_len = rows ? rows[g].q3.y : lv.axes[2 * g + 1];
        const float pa = a_len * ((hx * yx + hy * yy) + hz * yz);
        const float pb = b_len * ((bhx * yx + bhy * yy) + bhz * yz);
        float W = sqrtf(pa * pa + pb * pb);
        if (!(pl > 1e-7f)) W = fmaxf(a_len, b_len);
        hw = W / gr.s;
    }
    SegRec r;
    r.xa = (int)rintf((dot_e(gr.b.e1, ax, ay, az) - gr.u0) * gr.k16);
    r.ya = (int)rintf((dot_e(gr.b.e2, ax, ay, az) - gr.v0) * gr.k16);
    r.xb = (int)rintf((dot_e(gr.b.e1, bx, by, bz) - gr.u0) * gr.k16);
    r.yb = (int)rintf((dot_e(gr.b.e2, bx, by, bz) - gr.v0) * gr.k16);
    r.iza = gr.z_ref - dot_e(gr.b.d, ax, ay, az);
    r.izb = gr.z_ref - dot_e(gr.b.d, bx, by, bz);
    r.hw = hw;
    const float hw16 = 16.0f * hw;
    r.hwfx = 0;
    if (isfinite(hw16) && hw16 >= 0.0f) {
        const float c16 = ceilf(hw16);
        if (abs(r.xb - r.xa) > kMaxAxis || abs(r.yb - r.ya) > kMaxAxis || c16 > (float)kMaxHwFx)
            r.hwfx = kFlagCulledLong;
        else
            r.hwfx = (int)c16 | kFlagVisible;
    }
    seg[g] = r;
}

__device__ inline float dom_fragment_count(const SegRec& s, const LevelDev& lv, const ShadeRec* rows, float s_tex,
                                           uint32_t g, int px, int py);

// Per texel (one block per 16 x 16 tile): the first hit iz0 (the pixel's smallest key), then
// every fragment's expected hair count into its layer floor((iz0 - iz) / delta) (clamped to
// K - 1): a strand its box coverage alpha, a thick hair alpha rho kappa l_max sqrt(1 - h^2)
// (Sec. 4, hair number; the chord along the light at the texel's offset h = delta / hw).
// One block per batch of whole texels (the camera pass's batches), one lane per fragment; the
// counts are summed per (texel, layer) in LDS.  Texels in no batch hold no hair (cleared).
// Output: (iz0, C_0 .. C_{K-1}) with C the cumulative counts; iz0 = 0 marks a texel without hair.
__device__ inline float dom_fragment_count(const SegRec& s, const LevelDev& lv, const ShadeRec* rows, float s_tex,
                                           uint32_t g, int px, int py) {
    const int ex = 16 * px + 8 - s.xa, ey = 16 * py + 8 - s.ya;
    const int dx = s.xb - s.xa, dy = s.yb - s.ya;
    const int tden = dx * dx + dy * dy, cr = ex * dy - ey * dx;
    const float dl = fabsf((float)cr) / sqrtf((float)tden) * (1.0f / 16.0f);
    const float hw = s.hw;
    float c = fminf(fmaxf(fminf(dl + hw, 0.5f) - fmaxf(dl - hw, -0.5f), 0.0f), 1.0f);
    const bool thick = rows ? !row_is_strand(rows[g]) : lv.kind != 0;
    if (thick && !(hw > 0.0f)) {
        c = 0.0f;   // a degenerate (zero-width) thick hair holds no hairs across the light
    } else if (thick) {
        const int owner = g / lv.S;
        const float a = rows ? rows[g].q3.x : lv.axes[2 * g], b = rows ? rows[g].q3.y : lv.axes[2 * g + 1];
        const float n = rows ? rows[g].q3.z : (float)lv.n_total[owner], r = rows ? rows[g].q3.w : lv.r[owner];
        const float h = fminf(dl / hw, 1.0f);
        const float rho = fminf(fmaxf(n * r * r / (a * b), 0.0f), 1.0f);
        const float kappa = sqrtf(n / (3.14159265358979f * a * b));
        c = c * rho * kappa * (2.0f * a * b / (hw * s_tex)) * sqrtf((1.0f - h) * (1.0f + h));
    }
    return c;
}

__global__ __launch_bounds__(kNT) void k_dom_resolve(FrameBufs f, LevelDev lv, const ShadeRec* __restrict__ rows,
                                                     const DomGrid* __restrict__ grid, int K, float delta,
                                                     float4* __restrict__ tex) {
    // per (texel, layer) sums in 32.32 fixed point: integer adds commute, so the LDS atomics
    // give the same sums in any order (counts are far below 2^31 hairs; resolution 2^-32)
    __shared__ unsigned long long s_acc[kDomMaxLayers][kTilePix];
    __shared__ float s_iz0[kTilePix];
    const uint32_t n_batches = f.batch_start[f.T];
    const uint4 br = f.batches[blockIdx.x];
    if (blockIdx.x >= n_batches || f.ctr->cap_overflow) return;
    const BatchRec b = unpack_batch(br);
    const int tile = b.tile, p0 = b.p0, p1 = b.p1;
    const int t = threadIdx.x;
    const int R = grid->R;
    const float s_tex = grid->s;
    const int tx0 = (tile % f.ntx) * kTile, ty0 = (tile / f.ntx) * kTile;
    const size_t q = (size_t)tile * kTilePix + t;
    const bool mine = t >= p0 && t < p1;
    s_iz0[t] = (mine && f.pix_cnt[q]) ? __uint_as_float(0xFFFFFFFFu - f.pix_kmin[q]) : 0.0f;
#pragma unroll
    for (int k = 0; k < kDomMaxLayers; ++k) s_acc[k][t] = 0ull;
    __syncthreads();
    const uint2* fr = f.frags + b.frag0;
    const uint32_t* list = f.list + f.tile_start[tile];
    // kU records per lane in flight: the record, list and segment gathers of one round are
    // issued together instead of one dependent chain per record
    constexpr int kU = 4;
    for (uint32_t i0 = 0; i0 < b.nfrag; i0 += kU * kNT) {
        uint2 rec[kU];
        uint32_t g[kU];
        SegRec sg[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + t + u * kNT;
            rec[u] = i < b.nfrag ? fr[i] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + t + u * kNT;
            g[u] = i < b.nfrag ? seg_of(rec[u].y, list, f.gid != 0) : 0u;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + t + u * kNT;
            if (i < b.nfrag) sg[u] = f.seg[g[u]];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + t + u * kNT;
            if (i >= b.nfrag) continue;
            const uint32_t p = rec[u].y >> 24;
            const float iz = __uint_as_float(0xFFFFFFFFu - rec[u].x);
            const int layer = min(K - 1, (int)floorf((s_iz0[p] - iz) / delta));
            const float c = dom_fragment_count(sg[u], lv, rows, s_tex, g[u], tx0 + (int)(p % kTile), ty0 + (int)(p / kTile));
            const unsigned long long fx = (unsigned long long)((double)c * 4294967296.0 + 0.5);
            if (fx) atomicAdd(&s_acc[layer][p], fx);
        }
    }
    __syncthreads();
    const int px = tx0 + (t % kTile), py = ty0 + (t / kTile);
    if (!mine || px >= R || py >= R) return;
    float C[kDomMaxLayers];
    unsigned long long run = 0;
#pragma unroll
    for (int k = 0; k < kDomMaxLayers; ++k) {
        run += s_acc[k][t];
        C[k] = (float)((double)run * (1.0 / 4294967296.0));
    }
    const size_t o = 2 * ((size_t)py * R + px);
    tex[o] = make_float4(s_iz0[t], C[0], C[1], C[2]);
    tex[o + 1] = make_float4(C[3], C[4], C[5], C[6]);
}
}  // namespace

// ---------------------------------------------------------------------------------------
hipError_t launch_project(const LevelDev& lv, const CamConst& cam, SegRec* seg, ShadeRec* shade, hipStream_t st) {
    if (lv.nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project, dim3(blocks_for(lv.nseg, 256)), dim3(256), 0, st, lv, cam, seg, shade);
    return hipGetLastError();
}

hipError_t launch_tess(const LevelDev& lv, const CamConst& cam, int32_t max_px, int32_t max_sub, uint32_t* cnt,
                       uint32_t* start, uint32_t* scan_tmp, hipStream_t st) {
    if (lv.nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tess_count, dim3(blocks_for(lv.nseg, 256)), dim3(256), 0, st, lv, cam, 16 * max_px, max_sub,
                       cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_exscan(cnt, start, lv.nseg, scan_tmp, st);
}

hipError_t launch_tess_fill(const uint32_t* cnt, const uint32_t* start, int32_t nseg, uint32_t* rows, hipStream_t st) {
    if (nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tess_fill, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, cnt, start, nseg, rows);
    return hipGetLastError();
}

hipError_t launch_split(const LevelDev& lv, const CamConst& cam, uint32_t* cnt, uint32_t* start, uint32_t* scan_tmp,
                        hipStream_t st) {
    if (lv.nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_count, dim3(blocks_for(lv.nseg, 256)), dim3(256), 0, st, lv, cam, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_exscan(cnt, start, lv.nseg, scan_tmp, st);
}

hipError_t launch_split_mixed(const HierDev& h, const uint32_t* sel, int32_t nsel, const CamConst& cam, uint32_t* cnt,
                              uint32_t* start, uint32_t* scan_tmp, hipStream_t st) {
    if (nsel == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_count_mixed, dim3(blocks_for(nsel, 256)), dim3(256), 0, st, h, sel, nsel, cam, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_exscan(cnt, start, nsel, scan_tmp, st);
}

hipError_t launch_project_split_mixed(const HierDev& h, const uint32_t* sel, const uint32_t* rows, int32_t nrows,
                                      const uint32_t* cnt, const CamConst& cam, SegRec* seg, ShadeRec* shade,
                                      hipStream_t st) {
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project_split_mixed, dim3(blocks_for(nrows, 256)), dim3(256), 0, st, h, sel, rows, nrows, cnt,
                       cam, seg, shade);
    return hipGetLastError();
}

hipError_t launch_split_fill(const uint32_t* cnt, const uint32_t* start, int32_t nseg, uint32_t* rows, hipStream_t st) {
    if (nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_fill, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, cnt, start, nseg, rows);
    return hipGetLastError();
}

hipError_t launch_project_split(const LevelDev& lv, const uint32_t* rows, int32_t nrows, const uint32_t* cnt,
                                const CamConst& cam, SegRec* seg, ShadeRec* shade, hipStream_t st) {
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project_split, dim3(blocks_for(nrows, 256)), dim3(256), 0, st, lv, rows, nrows, cnt, cam, seg,
                       shade);
    return hipGetLastError();
}

hipError_t launch_project_tess(const LevelDev& lv, const uint32_t* rows, int32_t nrows, const uint32_t* cnt,
                               const CamConst& cam, SegRec* seg, ShadeRec* shade, hipStream_t st) {
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project_tess, dim3(blocks_for(nrows, 256)), dim3(256), 0, st, lv, rows, nrows, cnt, cam, seg,
                       shade);
    return hipGetLastError();
}

int dom_bound_blocks(int32_t nseg) {
    return std::max(1, std::min(kDomBoundMaxBlocks, (int)((nseg + kDomBoundThreads - 1) / kDomBoundThreads)));
}

hipError_t launch_dom_grid(const LevelDev& lv, const ShadeRec* rows, const DomBasis& b, int32_t R, float* part,
                           DomGrid* grid, hipStream_t st) {
    const int nb = dom_bound_blocks(lv.nseg);
    hipLaunchKernelGGL(k_dom_bounds, dim3(nb), dim3(kDomBoundThreads), 0, st, lv, rows, b, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dom_grid, dim3(1), dim3(kDomBoundThreads), 0, st, part, nb, b, R, grid);
    return hipGetLastError();
}

hipError_t launch_project_light(const LevelDev& lv, const ShadeRec* rows, const DomGrid* grid, SegRec* seg,
                                hipStream_t st) {
    if (lv.nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project_light, dim3(blocks_for(lv.nseg, 256)), dim3(256), 0, st, lv, rows, grid, seg);
    return hipGetLastError();
}

hipError_t launch_dom_resolve(const FrameBufs& f, const LevelDev& lv, const ShadeRec* rows, const DomGrid* grid,
                              int32_t K, float delta, int32_t R, uint32_t n_batches, float4* tex, hipStream_t st) {
    // n_batches: the grid (at least the frame's batch count, which the kernel reads)
    hipError_t e = launch_fill_f32(reinterpret_cast<float*>(tex), 0.0f, 8ull * R * R, st);
    if (e != hipSuccess || n_batches == 0) return e;
    hipLaunchKernelGGL(k_dom_resolve, dim3(n_batches), dim3(kNT), 0, st, f, lv, rows, grid, K, delta, tex);
    return hipGetLastError();
}

BinPlan bin_plan(int32_t nseg, int32_t T) {
    BinPlan p;
    p.range = std::min(T, kMaxLdsTiles);
    const int bytes = 4 * p.range;
    const int per_cu = std::max(1, std::min(2, (160 * 1024) / (bytes + 2048)));
    long nb = 256L * per_cu;
    nb = std::min(nb, std::max(32L, (long)((1 << 24) / std::max(T, 1))));
    nb = std::min(nb, std::max(1L, (long)((nseg + kBinThreads - 1) / kBinThreads)));
    p.nb = (int)std::max(1L, nb);
    p.per_block = (nseg + p.nb - 1) / p.nb;
    return p;
}

// Dynamic LDS above 64 KiB is declared to the runtime first (gfx950 has 160 KiB per CU); a
// runtime that needs no declaration may refuse the call, and the launch itself then decides.
static hipError_t allow_lds(const void* fn, int bytes) {
    if (bytes > 64 * 1024 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
        (void)hipGetLastError();
    return hipSuccess;
}

hipError_t launch_bins(const SegRec* seg, int32_t nseg, const CamConst& cam, const BinPlan& p, uint32_t* M,
                       uint4* blk, uint32_t* tot, uint32_t* tile_start, Counters* ctr, uint32_t* scan_tmp,
                       hipStream_t st) {
    const int ntx = (cam.W + kTile - 1) / kTile, nty = (cam.H + kTile - 1) / kTile, T = ntx * nty;
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_bin_count), 4 * p.range);
    if (e != hipSuccess) return e;
    for (int t0 = 0; t0 < T; t0 += p.range) {
        const int nt = std::min(p.range, T - t0);
        hipLaunchKernelGGL(k_bin_count, dim3(p.nb), dim3(kBinThreads), 4 * nt, st, seg, nseg, p.per_block, ntx, nty,
                           t0, nt, M, blk);
    }
    hipLaunchKernelGGL(k_bin_offsets, dim3(blocks_for(T, 64)), dim3(1024), 0, st, M, p.nb, T, tot, blk, ctr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_exscan(tot, tile_start, T, scan_tmp, st);
}

hipError_t launch_exscan(const uint32_t* cnt, uint32_t* start, int32_t n, uint32_t* scratch, hipStream_t st) {
    if (n <= kScanOneBlock) {
        hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, st, cnt, start, n);
        return hipGetLastError();
    }
    const int nb = (n + kScanChunk - 1) / kScanChunk;
    uint32_t* part = scratch;            // [nb]
    uint32_t* base = scratch + nb + 1;   // [nb + 1]
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(1024), 0, st, cnt, start, part, n);
    hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, st, part, base, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, st, start, base, n, nb);
    return hipGetLastError();
}

hipError_t launch_scatter(const SegRec* seg, int32_t nseg, const CamConst& cam, const BinPlan& p,
                          const uint32_t* tile_start, const uint32_t* M, uint32_t* list, const Counters* ctr,
                          hipStream_t st) {
    if (nseg == 0) return hipSuccess;
    const int ntx = (cam.W + kTile - 1) / kTile, nty = (cam.H + kTile - 1) / kTile, T = ntx * nty;
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_scatter), 4 * p.range);
    if (e != hipSuccess) return e;
    for (int t0 = 0; t0 < T; t0 += p.range) {
        const int nt = std::min(p.range, T - t0);
        hipLaunchKernelGGL(k_scatter, dim3(p.nb), dim3(kBinThreads), 4 * nt, st, seg, nseg, p.per_block, ntx, nty, t0,
                           nt, tile_start, M, list, ctr);
    }
    return hipGetLastError();
}

hipError_t launch_items_scan(const uint32_t* tile_start, int T, uint32_t* item_start, Counters* ctr,
                             uint32_t cap_pairs, uint32_t cap_items, hipStream_t st) {
    hipLaunchKernelGGL(k_items_scan, dim3(1), dim3(1024), 0, st, tile_start, T, item_start, ctr, cap_pairs, cap_items);
    return hipGetLastError();
}

hipError_t launch_tile_scans(const FrameBufs& f, uint32_t* frag_base, uint32_t* batch_start, uint32_t cap_frags,
                             uint32_t cap_batches, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_scans, dim3(1), dim3(1024), 0, st, f.tile_tot, frag_base, f.tile_nb, batch_start, f.T,
                       f.ctr, cap_frags, cap_batches);
    return hipGetLastError();
}

hipError_t launch_tile_items(const uint32_t* tile_start, int T, uint32_t* items, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_items, dim3(blocks_for(T, 256)), dim3(256), 0, st, tile_start, T, items);
    return hipGetLastError();
}

hipError_t launch_count(const FrameBufs& f, const CamConst& cam, uint32_t grid, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(kNT), 0, st, f, cam);
    return hipGetLastError();
}

hipError_t launch_tile_prep(const FrameBufs& f, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_prep, dim3(f.T), dim3(kNT), 0, st, f);
    return hipGetLastError();
}

hipError_t launch_batch_records(const FrameBufs& f, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_records, dim3(f.T), dim3(kNT), 0, st, f);
    return hipGetLastError();
}

hipError_t launch_emit(const FrameBufs& f, const CamConst& cam, uint32_t grid, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    if (f.pix_thick) hipLaunchKernelGGL(k_emit<true>, dim3(grid), dim3(kNT), 0, st, f, cam);
    else hipLaunchKernelGGL(k_emit<false>, dim3(grid), dim3(kNT), 0, st, f, cam);
    return hipGetLastError();
}

hipError_t launch_batches(const FrameBufs& f, const LevelDev& lv, const CamConst& cam, const LightsConst& lights,
                          const MatConst& mat, uint32_t n_batches, float* rgba, const DebugDump* dbg, hipStream_t st) {
    // n_batches: the grid (at least the frame's batch count, which the kernels read)
    if (n_batches == 0) return hipSuccess;
    ShadeArgs a;
    a.cam = cam;
    a.lights = lights;
    a.mat = mat;
    a.seg = f.seg;
    a.shade = f.shade;
    DebugDump d = dbg ? *dbg : DebugDump{};
    const int hd = dbg ? 1 : 0;
    const dim3 g(n_batches), b(kNT);
    bool shadow = false;
    for (int i = 0; i < lights.n; ++i) shadow |= lights.dom[i].grid != nullptr;
    if (lv.kind != 2) {
        if (shadow) {
            if (mat.model == 0) {
                if (lv.kind == 0) hipLaunchKernelGGL((k_batch<0, 0, true>), g, b, 0, st, f, a, rgba, d, hd);
                else hipLaunchKernelGGL((k_batch<1, 0, true>), g, b, 0, st, f, a, rgba, d, hd);
            } else {
                if (lv.kind == 0) hipLaunchKernelGGL((k_batch<0, 1, true>), g, b, 0, st, f, a, rgba, d, hd);
                else hipLaunchKernelGGL((k_batch<1, 1, true>), g, b, 0, st, f, a, rgba, d, hd);
            }
        } else if (mat.model == 0) {
            if (lv.kind == 0) hipLaunchKernelGGL((k_batch<0, 0, false>), g, b, 0, st, f, a, rgba, d, hd);
            else hipLaunchKernelGGL((k_batch<1, 0, false>), g, b, 0, st, f, a, rgba, d, hd);
        } else {
            if (lv.kind == 0) hipLaunchKernelGGL((k_batch<0, 1, false>), g, b, 0, st, f, a, rgba, d, hd);
            else hipLaunchKernelGGL((k_batch<1, 1, false>), g, b, 0, st, f, a, rgba, d, hd);
        }
        return hipGetLastError();
    }
    // A mixed frame: the strand-only batches (KIND 3), then those holding thick-hair fragments
    // (KIND 2); the kernels choose between them on the device (see k_batch).
    if (shadow) {
        if (mat.model == 0) {
            hipLaunchKernelGGL((k_batch<3, 0, true>), g, b, 0, st, f, a, rgba, d, hd);
            hipLaunchKernelGGL((k_batch<2, 0, true>), g, b, 0, st, f, a, rgba, d, hd);
        } else {
            hipLaunchKernelGGL((k_batch<3, 1, true>), g, b, 0, st, f, a, rgba, d, hd);
            hipLaunchKernelGGL((k_batch<2, 1, true>), g, b, 0, st, f, a, rgba, d, hd);
        }
    } else if (mat.model == 0) {
        hipLaunchKernelGGL((k_batch<3, 0, false>), g, b, 0, st, f, a, rgba, d, hd);
        hipLaunchKernelGGL((k_batch<2, 0, false>), g, b, 0, st, f, a, rgba, d, hd);
    } else {
        hipLaunchKernelGGL((k_batch<3, 1, false>), g, b, 0, st, f, a, rgba, d, hd);
        hipLaunchKernelGGL((k_batch<2, 1, false>), g, b, 0, st, f, a, rgba, d, hd);
    }
    return hipGetLastError();
}

hipError_t launch_lod_init(const HierDev& h, const CamConst& cam, float eps_w, int32_t* levels, hipStream_t st) {
    const int gk = h.G * h.S;
    if (gk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lod_init, dim3((gk + 3) / 4), dim3(256), 0, st, h, cam, eps_w, levels);
    return hipGetLastError();
}

hipError_t launch_lod_update(const HierDev& h, const CamConst& cam, float eps_w, int32_t* levels, hipStream_t st) {
    const int gk = h.G * h.S;
    if (gk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lod_update, dim3((gk + 3) / 4), dim3(256), 0, st, h, cam, eps_w, levels);
    return hipGetLastError();
}

hipError_t launch_select(const HierDev& h, const int32_t* levels, uint32_t* cnt, uint32_t* sel_start,
                         uint32_t* scan_tmp, hipStream_t st) {
    const int gk = h.G * h.S;
    hipLaunchKernelGGL(k_sel_count, dim3(blocks_for(gk, 256)), dim3(256), 0, st, h, levels, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_exscan(cnt, sel_start, gk, scan_tmp, st);
}

hipError_t launch_select_fill(const HierDev& h, const int32_t* levels, const uint32_t* sel_start, uint32_t* sel,
                              hipStream_t st) {
    const int gk = h.G * h.S;
    hipLaunchKernelGGL(k_sel_fill, dim3((gk + 3) / 4), dim3(256), 0, st, h, levels, sel_start, sel);
    return hipGetLastError();
}

hipError_t launch_project_mixed(const HierDev& h, const uint32_t* sel, int32_t nsel, const CamConst& cam, SegRec* seg,
                                ShadeRec* shade, hipStream_t st) {
    if (nsel == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project_mixed, dim3(blocks_for(nsel, 256)), dim3(256), 0, st, h, sel, nsel, cam, seg, shade);
    return hipGetLastError();
}

hipError_t launch_batches_bwd(const FrameBufs& f, const LevelDev& lv, const CamConst& cam, const LightsConst& lights,
                              const MatConst& mat, uint32_t n_batches, const GradOut& grad, hipStream_t st) {
    if (n_batches == 0) return hipSuccess;
    ShadeArgs a;
    a.cam = cam;
    a.lights = lights;
    a.mat = mat;
    a.seg = f.seg;
    a.shade = f.shade;
    if (mat.model == 0)
        hipLaunchKernelGGL(k_batch_bwd<0>, dim3(n_batches), dim3(kNT), 0, st, f, a, grad, lv.S, lv.n_owner);
    else
        hipLaunchKernelGGL(k_batch_bwd<1>, dim3(n_batches), dim3(kNT), 0, st, f, a, grad, lv.S, lv.n_owner);
    return hipGetLastError();
}

hipError_t launch_build_centers(const float* vx, const float* vy, const float* vz, const float* width, const float* sig,
                                int32_t n_strands, int32_t V, const int32_t* members, const int32_t* member_start,
                                int32_t K, float* cx, float* cy, float* cz, float* r, float* csig, int32_t* n_total,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_build_centers, dim3(blocks_for((size_t)K * V, 128)), dim3(128), 0, st, vx, vy, vz, width, sig,
                       n_strands, V, members, member_start, K, cx, cy, cz, r, csig, n_total);
    return hipGetLastError();
}

hipError_t launch_build_ellipses(const float* vx, const float* vy, const float* vz, int32_t V, const int32_t* members,
                                 const int32_t* member_start, int32_t K, const float* cx, const float* cy,
                                 const float* cz, const float* r, float* ahat, float* axes, hipStream_t st) {
    hipLaunchKernelGGL(k_build_ellipses, dim3(blocks_for((size_t)K * (V - 1), 128)), dim3(128), 0, st, vx, vy, vz, V,
                       members, member_start, K, cx, cy, cz, r, ahat, axes);
    return hipGetLastError();
}

hipError_t launch_check_caps(const FrameBufs& f, const FrameCaps& caps, int stage, hipStream_t st) {
    hipLaunchKernelGGL(k_check_caps, dim3(1), dim3(64), 0, st, f, caps, stage);
    return hipGetLastError();
}

hipError_t launch_fill_pix(uint32_t* cnt, uint32_t* kmin, uint32_t* kmax, uint8_t* thick, size_t n, float* rgba,
                           size_t n_rgba4, const uint32_t* item_start, int T, uint2* item_tab, uint32_t cap_items,
                           hipStream_t st) {
    const size_t m = std::max(std::max(n, n_rgba4), (size_t)T * 64);
    if (m == 0) return hipSuccess;
    const int nb = (int)std::min<size_t>((m + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_pix, dim3(nb), dim3(256), 0, st, cnt, kmin, kmax, thick, n,
                       reinterpret_cast<float4*>(rgba), rgba ? n_rgba4 : 0, item_start, T, item_tab, cap_items);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// Issue-rate probe: every lane runs `iters` rounds of 8 independent chains of one instruction
// (0: v_fma_f32, 1: v_exp_f32, 2: v_rcp_f32, 3: v_sqrt_f32, 4: v_mul_lo_u32, 5: v_mul_u32_u24),
// so that the rate, not the latency, bounds the kernel.  The chains stay finite and bounded
// (exp2 of a value in [-1, 0], rcp alternating, sqrt toward 1, integer products wrapping);
// their sum is stored only if it equals an impossible value, which keeps them live.
template <int KIND>
__global__ __launch_bounds__(256) void k_probe_rate(float* __restrict__ out, int iters) {
    float a[8];
    uint32_t u[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = 0.5f + 1e-3f * (float)(threadIdx.x & 63) + 0.01f * (float)i;
        u[i] = threadIdx.x * 8u + (uint32_t)i + 1u;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (KIND == 0) a[i] = __builtin_fmaf(a[i], 0.999f, 1e-4f);
            if (KIND == 1) a[i] = __builtin_amdgcn_exp2f(-a[i]);
            if (KIND == 2) a[i] = __builtin_amdgcn_rcpf(a[i]);
            if (KIND == 3) a[i] = __builtin_amdgcn_sqrtf(a[i]);
            if (KIND == 4) u[i] = u[i] * 0x9E3779B1u;
            if (KIND == 5) u[i] = __umul24(u[i], 0x3779B1u);
        }
    }
    float sum = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) sum += a[i] + (float)u[i];
    if (sum == -1.0f) out[0] = sum;
}

hipError_t launch_probe_rate(int kind, int blocks, int iters, float* out, hipStream_t st) {
    switch (kind) {
        case 0: hipLaunchKernelGGL(k_probe_rate<0>, dim3(blocks), dim3(256), 0, st, out, iters); break;
        case 1: hipLaunchKernelGGL(k_probe_rate<1>, dim3(blocks), dim3(256), 0, st, out, iters); break;
        case 2: hipLaunchKernelGGL(k_probe_rate<2>, dim3(blocks), dim3(256), 0, st, out, iters); break;
        case 3: hipLaunchKernelGGL(k_probe_rate<3>, dim3(blocks), dim3(256), 0, st, out, iters); break;
        case 4: hipLaunchKernelGGL(k_probe_rate<4>, dim3(blocks), dim3(256), 0, st, out, iters); break;
        default: hipLaunchKernelGGL(k_probe_rate<5>, dim3(blocks), dim3(256), 0, st, out, iters); break;
    }
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(min(blocks_for(n, 256), 4096)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace hair
