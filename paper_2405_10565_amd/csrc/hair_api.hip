// C-ABI of libhair.so: contexts with an HBM budget, resident assets and LoD levels,
// workspaces, host-side argument validation (always before any launch), and the frame
// orchestration around the kernels of hair_kernels.hip.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hair_internal.h"

using namespace hair;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    template <class T> T* as() const { return static_cast<T*>(p); }
};

struct Level {
    int K = 0, S = 0;
    DevBuf cx, cy, cz, ahat, axes, n_total, r, sig;
};

// Nested hierarchy for per-group level choice: groups = clusters of the coarsest level; per
// level l (0 = strands) its owners listed by group (CSR, ascending owner ids per group).
struct Hierarchy {
    bool nested = false;
    int G = 0;
    std::vector<DevBuf> grp_start, grp_owner;   // [n_levels + 1]
};

struct Asset {
    int n_strands = 0, V = 0, S = 0;
    DevBuf x, y, z, width, sig;
    hair_material mat{};
    std::vector<Level> levels;   // levels[l - 1] is level l
    Hierarchy hier;
};

// Static scratch of hair_render_noalloc: every device the library runs on holds one copy of
// it until the process ends.  In host code the name stands for a host-side shadow, not a
// device address; host code uses only the per-device address that hipGetSymbolAddress
// returned for it (scratch_ptr below).
constexpr size_t kScratchBytes = 64ull << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;   // device -> its copy of scratch

// The device's copy of scratch; the device must be current.  Looked up once per device.
hipError_t scratch_ptr(int device, unsigned char** out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<unsigned char*>(ptr);
    *out = static_cast<unsigned char*>(ptr);
    return hipSuccess;
}

bool finite_all(const float* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

struct hair_ctx {
    int device = -1;
    uint64_t budget = 0;
    uint64_t used = 0;
    bool poisoned = false;
    std::mutex mu;
    std::map<int, Asset> assets;
    int next_id = 1;
    hair_ws* default_ws = nullptr;
    hair_ws* fixed_ws = nullptr;   // frames of hair_render_noalloc (buffers in the static scratch)
};

struct hair_ws {
    hair_ctx* ctx = nullptr;
    uint64_t max_bytes = 0;
    uint64_t held = 0;
    DevBuf seg, shade, scan_tmp, tile_cnt, tile_start, bin_m, bin_blk, list, ctr, sel_cnt, sel_start, sel, sel_tmp;
    DevBuf pieces;                            // rows of a frame drawn with long segments as pieces
    DevBuf items, item_start, item_tab, item_base, pix_cnt, pix_kmin, pix_kmax, pix_off, pix_thick, thick_list;
    DevBuf tile_tot, frag_base, tile_nb, batch_mask, batch_start, batches, frags;
    DevBuf dom_tex, dom_grid, dom_part;      // shadow pass: texels, grids, bounds partials
    int32_t dom_R = 0, dom_K = 0, dom_n = 0;  // last shadowed render: resolution, layers, maps
    int32_t dom_light[HAIR_MAX_LIGHTS] = {};  // map index of each light, -1 if unshadowed
    FrameCaps caps = {};                      // buffer capacities of warm frames (0: none yet)
    hipEvent_t ev[7] = {};
    bool events = false;
    int64_t last_nseg = 0, last_ntiles = 0, last_pairs = 0;
    // a frame enqueued by hair_render_async and not yet finished: what a rerun needs, and
    // (done) the result of a frame that already ran to completion
    struct Pending {
        bool active = false, done = false;
        int32_t asset = -1, level = 0;
        hair_camera cam{};
        std::vector<hair_light> lights;
        float* rgba = nullptr;
        hipStream_t st = nullptr;
        Counters ctr{};            // result of a frame that ran to completion (done)
        uint32_t pairs = 0, n_batches = 0;
        float ms[4] = {};
    } pending;
    Counters* ctr_host = nullptr;   // pinned copy of a deferred frame's counters
    // A workspace over the device's static scratch (hair_render_noalloc): its buffers are
    // carved from [arena, arena + arena_bytes) afresh for every frame and never allocated.
    unsigned char* arena = nullptr;
    size_t arena_bytes = 0, arena_off = 0;
    std::mutex mu;
};

namespace {

int dev_fail(hair_ctx* ctx, hipError_t e, const char* what) {
    if (ctx) ctx->poisoned = true;
    return fail(HAIR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr, what)                      \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return dev_fail(ctx, _e, what); \
    } while (0)

int ctx_alloc(hair_ctx* ctx, DevBuf& b, size_t bytes, hair_ws* ws = nullptr) {
    if (bytes == 0) bytes = 4;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        if (ctx->used + bytes > ctx->budget)
            return fail(HAIR_ENOMEM, "allocation of %zu bytes exceeds the HBM budget (%llu of %llu used)", bytes,
                        (unsigned long long)ctx->used, (unsigned long long)ctx->budget);
        if (ws && ws->max_bytes && ws->held + bytes > ws->max_bytes)
            return fail(HAIR_ENOMEM, "workspace limit of %llu bytes exceeded", (unsigned long long)ws->max_bytes);
        ctx->used += bytes;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->used -= bytes;
        b.p = nullptr;
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            return fail(HAIR_ENOMEM, "device out of memory for %zu bytes", bytes);
        }
        return dev_fail(ctx, e, "hipMalloc");
    }
    b.bytes = bytes;
    if (ws) ws->held += bytes;
    return HAIR_OK;
}

void ctx_free(hair_ctx* ctx, DevBuf& b, hair_ws* ws = nullptr) {
    if (!b.p) return;
    (void)hipFree(b.p);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->used -= b.bytes;
    if (ws) ws->held -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
}

// Every device buffer a workspace can hold.
std::array<DevBuf*, 34> ws_buffers(hair_ws* ws) {
    return {{&ws->seg, &ws->shade, &ws->scan_tmp, &ws->tile_cnt, &ws->tile_start, &ws->bin_m, &ws->bin_blk,
            &ws->sel_cnt, &ws->sel_start, &ws->sel, &ws->sel_tmp, &ws->list, &ws->ctr, &ws->items,
            &ws->item_start, &ws->item_tab, &ws->item_base, &ws->pix_cnt, &ws->pix_kmin, &ws->pix_kmax, &ws->pix_off, &ws->pix_thick, &ws->thick_list,
            &ws->tile_tot, &ws->frag_base, &ws->tile_nb, &ws->batch_mask, &ws->batch_start, &ws->batches,
            &ws->frags, &ws->dom_tex, &ws->dom_grid, &ws->dom_part, &ws->pieces}};
}

// A buffer carved from a static-scratch workspace (256-byte aligned, no headroom).
int arena_take(hair_ws* ws, DevBuf& b, size_t bytes) {
    if (b.p && b.bytes >= bytes) return HAIR_OK;
    if (bytes == 0) bytes = 4;
    const size_t off = (ws->arena_off + 255) & ~size_t(255);
    if (bytes > ws->arena_bytes || off > ws->arena_bytes - bytes)
        return fail(HAIR_ENOMEM, "the frame needs more than the %zu bytes of static scratch of hair_render_noalloc",
                    ws->arena_bytes);
    b.p = ws->arena + off;
    b.bytes = bytes;
    ws->arena_off = off + bytes;
    return HAIR_OK;
}

// Grow-only workspace buffer (25% headroom).
int ws_need(hair_ws* ws, DevBuf& b, size_t bytes) {
    if (ws->arena) return arena_take(ws, b, bytes);
    if (b.bytes >= bytes && b.p) return HAIR_OK;
    ctx_free(ws->ctx, b, ws);
    return ctx_alloc(ws->ctx, b, bytes + bytes / 4 + 256, ws);
}

void free_level(hair_ctx* ctx, Level& l) {
    for (DevBuf* b : {&l.cx, &l.cy, &l.cz, &l.ahat, &l.axes, &l.n_total, &l.r, &l.sig}) ctx_free(ctx, *b);
}

void free_hierarchy(hair_ctx* ctx, Hierarchy& h) {
    for (DevBuf& b : h.grp_start) ctx_free(ctx, b);
    for (DevBuf& b : h.grp_owner) ctx_free(ctx, b);
    h.grp_start.clear();
    h.grp_owner.clear();
    h.nested = false;
    h.G = 0;
}

void free_asset(hair_ctx* ctx, Asset& a) {
    for (DevBuf* b : {&a.x, &a.y, &a.z, &a.width, &a.sig}) ctx_free(ctx, *b);
    for (Level& l : a.levels) free_level(ctx, l);
    a.levels.clear();
    free_hierarchy(ctx, a.hier);
}

int check_ctx(hair_ctx* ctx) {
    if (!ctx) return fail(HAIR_EINVAL, "null context");
    if (ctx->poisoned) return fail(HAIR_EDEVICE, "context poisoned by an earlier device error");
    return HAIR_OK;
}

int need_device(hair_ctx* ctx) {
    if (ctx->device < 0) return fail(HAIR_EDEVICE, "host-only context: no device work possible");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return dev_fail(ctx, e, "hipSetDevice");
    return HAIR_OK;
}

int validate_material(const hair_material* m) {
    if (!m) return fail(HAIR_EINVAL, "null material");
    if (m->model == HAIR_MODEL_RTTD) {
        if (!(std::isfinite(m->beta_r) && m->beta_r > 0.0f && m->beta_r < 2.0f))
            return fail(HAIR_EINVAL, "material beta_r must be in (0, 2)");
        if (!(std::isfinite(m->beta_tt) && m->beta_tt > 0.0f && m->beta_tt < 2.0f))
            return fail(HAIR_EINVAL, "material beta_tt must be in (0, 2)");
        if (!(std::isfinite(m->gamma_tt) && m->gamma_tt > 0.0f && m->gamma_tt < 4.0f))
            return fail(HAIR_EINVAL, "material gamma_tt must be in (0, 4)");
        for (int c = 0; c < 3; ++c) {
            const float v[3] = {m->a_r[c], m->a_tt[c], m->a_d[c]};
            for (float x : v)
                if (!(std::isfinite(x) && x >= 0.0f)) return fail(HAIR_EINVAL, "material attenuations must be >= 0");
            if ((double)v[0] + v[1] + v[2] > 1.0)
                return fail(HAIR_EINVAL, "material a_r + a_tt + a_d must be <= 1 in every channel");
        }
        return HAIR_OK;
    }
    if (m->model != HAIR_MODEL_RTTRT) return fail(HAIR_EINVAL, "unknown material model %d", (int)m->model);
    if (!(std::isfinite(m->eta) && m->eta > 1.0f)) return fail(HAIR_EINVAL, "material eta must be finite and > 1");
    if (!std::isfinite(m->alpha) || std::fabs(m->alpha) > 0.5f)
        return fail(HAIR_EINVAL, "material alpha must be finite with |alpha| <= 0.5 rad");
    if (!(std::isfinite(m->beta_m) && m->beta_m > 0.0f && m->beta_m < 2.0f))
        return fail(HAIR_EINVAL, "material beta_m must be in (0, 2)");
    if (!(std::isfinite(m->beta_n) && m->beta_n > 0.0f && m->beta_n < 4.0f))
        return fail(HAIR_EINVAL, "material beta_n must be in (0, 4)");
    return HAIR_OK;
}

int validate_camera(const hair_camera* c) {
    if (!c) return fail(HAIR_EINVAL, "null camera");
    if (!finite_all(c->pos, 3) || !finite_all(c->rot, 9)) return fail(HAIR_EINVAL, "camera pose not finite");
    if (!(std::isfinite(c->fx) && c->fx > 0 && std::isfinite(c->fy) && c->fy > 0))
        return fail(HAIR_EINVAL, "camera focal lengths must be finite and > 0");
    if (!(std::isfinite(c->cx) && std::isfinite(c->cy))) return fail(HAIR_EINVAL, "camera principal point not finite");
    if (!(std::isfinite(c->z_near) && c->z_near > 0)) return fail(HAIR_EINVAL, "camera z_near must be > 0");
    if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
        return fail(HAIR_EINVAL, "image size %dx%d outside [1, 16384]", c->width, c->height);
    return HAIR_OK;
}

int validate_lights(const hair_light* l, int n) {
    if (!l) return fail(HAIR_EINVAL, "null lights");
    if (n < 1 || n > HAIR_MAX_LIGHTS) return fail(HAIR_EINVAL, "n_lights %d outside [1, %d]", n, HAIR_MAX_LIGHTS);
    for (int i = 0; i < n; ++i) {
        if (l[i].kind != 0 && l[i].kind != 1) return fail(HAIR_EINVAL, "light %d: unknown kind %d", i, l[i].kind);
        if (!finite_all(l[i].vec, 3) || !finite_all(l[i].rgb, 3)) return fail(HAIR_EINVAL, "light %d not finite", i);
        for (int c = 0; c < 3; ++c)
            if (l[i].rgb[c] < 0) return fail(HAIR_EINVAL, "light %d: negative intensity", i);
        if (l[i].kind == 0) {
            const float n2 = l[i].vec[0] * l[i].vec[0] + l[i].vec[1] * l[i].vec[1] + l[i].vec[2] * l[i].vec[2];
            if (std::fabs(n2 - 1.0f) > 1e-3f) return fail(HAIR_EINVAL, "light %d: direction is not unit length", i);
        }
    }
    return HAIR_OK;
}

CamConst cam_const(const hair_camera* c) {
    CamConst k;
    memcpy(k.pos, c->pos, sizeof(k.pos));
    memcpy(k.rot, c->rot, sizeof(k.rot));
    k.fx = c->fx; k.fy = c->fy; k.cx = c->cx; k.cy = c->cy; k.z_near = c->z_near;
    k.W = c->width; k.H = c->height;
    return k;
}

LightsConst lights_const(const hair_light* l, int n) {
    LightsConst k;
    memset(&k, 0, sizeof(k));
    k.n = n;
    for (int i = 0; i < n; ++i) {
        k.l[i].kind = l[i].kind;
        memcpy(k.l[i].vec, l[i].vec, sizeof(k.l[i].vec));
        memcpy(k.l[i].rgb, l[i].rgb, sizeof(k.l[i].rgb));
    }
    return k;
}

MatConst mat_const(const hair_material& m) {
    MatConst k{};
    k.eta = m.eta;
    k.inv_eta2 = (float)(1.0 / ((double)m.eta * (double)m.eta));
    k.alpha_p[0] = m.alpha; k.alpha_p[1] = -0.5f * m.alpha; k.alpha_p[2] = -1.5f * m.alpha;
    k.beta_p[0] = m.beta_m; k.beta_p[1] = 0.5f * m.beta_m; k.beta_p[2] = 2.0f * m.beta_m;
    for (int p = 0; p < 3; ++p) {
        const double b = k.beta_p[p];
        k.g_amp[p] = (float)(0.5 / (b * std::sqrt(2.0 * M_PI)));
        k.g_k[p] = (float)(1.0 / (2.0 * b * b));
        k.g_k2[p] = (float)(M_LOG2E / (2.0 * b * b));
    }
    k.beta_n = m.beta_n;
    const double s = std::sqrt(3.0) * (double)m.beta_n / M_PI;
    k.s = (float)s;
    k.inv_s = (float)(1.0 / s);
    k.inv_s_l2 = (float)(M_LOG2E / s);
    k.n_norm = (float)(1.0 / (s * std::tanh(M_PI / (2.0 * s))));
    for (int p = 0; p < 3; ++p)
        k.mn_amp[p] = (float)(0.5 / ((double)k.beta_p[p] * std::sqrt(2.0 * M_PI)) / (s * std::tanh(M_PI / (2.0 * s))));
    const double lo = 1.0 / (1.0 + std::exp(M_PI / s)), hi = 1.0 / (1.0 + std::exp(-M_PI / s));
    k.cdf_lo = (float)lo;
    k.cdf_scale = (float)(1.0 / (hi - lo));
    k.model = m.model;
    if (m.model == HAIR_MODEL_RTTD) {
        const double bR = m.beta_r, bT = m.beta_tt, g = m.gamma_tt;
        const double b[2] = {bR, bT};
        for (int p = 0; p < 2; ++p) {
            k.d_amp[p] = (float)(0.5 / (b[p] * std::sqrt(2.0 * M_PI)));
            k.d_k2[p] = (float)(M_LOG2E / (2.0 * b[p] * b[p]));
            k.d_beta2[p] = (float)(b[p] * b[p]);
        }
        k.n_amp = (float)(1.0 / (g * std::sqrt(2.0 * M_PI)));
        k.n_k2 = (float)(M_LOG2E / (2.0 * g * g));
        k.gamma2 = (float)(g * g);
        // hemisphere masses: R and D split evenly; TT (about phi = pi) puts erf(pi / (2 sqrt2 g))
        // in front (|phi| > pi/2), the rest of its wrapped mass behind
        const double fT = std::erf(0.5 * M_PI / (std::sqrt(2.0) * g));
        const double bTm = std::erf(M_PI / (std::sqrt(2.0) * g)) - fT;
        double mR = 0.0, mT = 0.0;
        for (int c = 0; c < 3; ++c) {
            k.A[0][c] = m.a_r[c];
            k.A[1][c] = m.a_tt[c];
            k.A[2][c] = m.a_d[c];
            k.aF[c] = (float)(0.5 * m.a_r[c] + fT * m.a_tt[c] + 0.5 * m.a_d[c]);
            k.aB[c] = (float)(0.5 * m.a_r[c] + bTm * m.a_tt[c] + 0.5 * m.a_d[c]);
            mR += m.a_r[c] / 3.0;
            mT += m.a_tt[c] / 3.0;
        }
        // attenuation-weighted longitudinal variances of the R and TT mass in each hemisphere
        auto mean_var = [&](double wR, double wT) { return wR + wT > 0.0 ? (wR * bR * bR + wT * bT * bT) / (wR + wT) : 0.0; };
        k.var_f = (float)mean_var(0.5 * mR, fT * mT);
        k.var_b = (float)mean_var(0.5 * mR, bTm * mT);
    }
    return k;
}

int find_level(hair_ctx* ctx, int32_t asset, int32_t level, Asset** a_out, LevelDev* lv) {
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    Asset& a = it->second;
    if (level < 0 || level > (int)a.levels.size()) return fail(HAIR_ENOENT, "asset %d has no level %d", asset, level);
    *a_out = &a;
    memset(lv, 0, sizeof(*lv));
    lv->S = a.S;
    if (level == 0) {
        lv->kind = 0;
        lv->nseg = a.n_strands * a.S;
        lv->n_owner = a.n_strands;
        lv->vx = a.x.as<float>(); lv->vy = a.y.as<float>(); lv->vz = a.z.as<float>();
        lv->width = a.width.as<float>();
        lv->sig = a.sig.as<float>();
    } else {
        Level& l = a.levels[level - 1];
        lv->kind = 1;
        lv->nseg = l.K * l.S;
        lv->n_owner = l.K;
        lv->vx = l.cx.as<float>(); lv->vy = l.cy.as<float>(); lv->vz = l.cz.as<float>();
        lv->sig = l.sig.as<float>();
        lv->ahat = l.ahat.as<float>();
        lv->axes = l.axes.as<float>();
        lv->n_total = l.n_total.as<int32_t>();
        lv->r = l.r.as<float>();
    }
    return HAIR_OK;
}

hair_ws* ws_or_default(hair_ctx* ctx, hair_ws* ws) {
    if (ws) return ws;
    std::lock_guard<std::mutex> g(ctx->mu);
    if (!ctx->default_ws) {
        ctx->default_ws = new hair_ws();
        ctx->default_ws->ctx = ctx;
    }
    return ctx->default_ws;
}

int ws_events(hair_ws* ws) {
    if (ws->events) return HAIR_OK;
    // ev[0], ev[5], ev[6] time the frame; ev[1] only marks a deferred frame's end (no timestamp)
    for (int i = 0; i < 7; ++i)
        HIP_TRY(ws->ctx, i == 1 ? hipEventCreateWithFlags(&ws->ev[i], hipEventDisableTiming) : hipEventCreate(&ws->ev[i]),
                "hipEventCreate");
    ws->events = true;
    return HAIR_OK;
}

struct FrameOut {
    Counters ctr;
    uint32_t pairs;
    uint32_t n_batches;
    float ms[4];
    bool deferred = false;   // counters and timings are read when the workspace is finished
};

// A frame's sizes and timings from its counters (after its stream has passed ev[6]).
int frame_result(hair_ctx* ctx, hair_ws* ws, int64_t nseg, int T, FrameOut* out) {
    const uint32_t pairs = out->ctr.sizes[0];
    ws->last_nseg = nseg;
    ws->last_ntiles = T;
    ws->last_pairs = pairs;
    out->pairs = pairs;
    out->ctr.fragments = out->ctr.sizes[2];
    out->n_batches = out->ctr.sizes[3];
    // three timing markers only: each costs the stream a few microseconds of idle time
    float t05 = 0, t56 = 0, t06 = 0;
    HIP_TRY(ctx, hipEventElapsedTime(&t05, ws->ev[0], ws->ev[5]), "elapsed");
    HIP_TRY(ctx, hipEventElapsedTime(&t56, ws->ev[5], ws->ev[6]), "elapsed");
    HIP_TRY(ctx, hipEventElapsedTime(&t06, ws->ev[0], ws->ev[6]), "elapsed");
    out->ms[0] = t06; out->ms[1] = t05; out->ms[2] = 0.0f; out->ms[3] = t56;
    return HAIR_OK;
}

// A shadow-pass raster: the light view's records instead of the camera's, and the per-texel
// layers instead of shading.
// A curved thick-hair frame: the row list over the level's segments (base) and their steps.
// A frame of pieces of the level's long segments (split): the same, with rows of pieces.
struct TessPass {
    LevelDev base;
    const uint32_t* rows;
    const uint32_t* cnt;
    bool split = false;
};

struct DomPass {
    const DomGrid* grid;
    int32_t K;
    float delta;
    float4* tex;
    const ShadeRec* rows;   // a mixed frame's rows (their camera shading records), or nullptr
};

// Project + bin + tile for one level; the caller holds ws->mu.
//   k_project                         per-segment records (projection, half-width, culling)
//   k_bin_count, k_bin_offsets, k_scan per-block tile counts, their column scan, list offsets
//   k_tile_items, k_scan              work items (list chunks) per tile
//   k_scatter                         tile lists (per-block LDS cursors)
//   k_count, k_tile_prep, k_scan x2   per-pixel counts, offsets, batches
//   k_batch_records, k_emit           batch table, fragment buffer and per-pixel key ranges
//   k_batch                           sort, shade, blend (one workgroup per batch)
// A cold frame reads the frame's sizes back twice (after the work items and after the
// batches) to size its buffers, with a quarter of headroom that the workspace keeps as its
// capacities.  A warm frame launches on those capacities without reading anything back: the
// kernels take the real sizes from device memory, k_check_caps flags a size beyond its
// capacity (after which the passes that fill sized buffers do nothing), and a flagged frame
// is rendered again cold.  The frame ends with one synchronisation for the counters.
static uint32_t with_headroom(uint32_t n) { return n + n / 4 + 256; }

int run_frame(hair_ctx* ctx, hair_ws* ws, const Asset& a, const LevelDev& lv, const hair_camera* cam,
              const hair_light* lights, int n_lights, float* rgba, const DebugDump* dbg, hipStream_t st,
              FrameOut* out, bool tiles_too = true, const GradOut* grad = nullptr, const HierDev* hier = nullptr,
              const uint32_t* sel = nullptr, const DomPass* dom = nullptr, const DomView* views = nullptr,
              const TessPass* tess = nullptr, bool cold = false, bool defer = false) {
    int rc;
    if (ws->pending.active)
        return fail(HAIR_EINVAL, "the workspace holds a frame of hair_render_async: call hair_ws_finish first");
    const CamConst cc = cam_const(cam);
    const int ntx = (cam->width + kTile - 1) / kTile, nty = (cam->height + kTile - 1) / kTile;
    const int T = ntx * nty;
    const size_t TP = (size_t)T * kTilePix;
    const BinPlan plan = bin_plan(lv.nseg, T);
    if (ws->arena) {   // static scratch: every frame is sized afresh from its own counts
        for (DevBuf* b : ws_buffers(ws)) *b = DevBuf{};
        ws->arena_off = 0;
        ws->caps = FrameCaps{};
    }
    const bool warm = tiles_too && !cold && !ws->arena && ws->caps.items > 0 && ws->caps.batches > 0;
    // with_headroom for buffers a workspace keeps; exact sizes in the static scratch
    auto cap_of = [&](uint32_t n) { return ws->arena ? n : with_headroom(n); };
    if ((rc = ws_events(ws))) return rc;
    if ((rc = ws_need(ws, ws->seg, sizeof(SegRec) * (size_t)std::max(lv.nseg, 1)))) return rc;
    if ((rc = ws_need(ws, ws->shade, sizeof(ShadeRec) * (size_t)std::max(lv.nseg, 1)))) return rc;
    if ((rc = ws_need(ws, ws->scan_tmp, 4 * exscan_scratch_words(T)))) return rc;
    if ((rc = ws_need(ws, ws->tile_cnt, 4ull * T))) return rc;
    if ((rc = ws_need(ws, ws->tile_start, 4ull * (T + 1)))) return rc;
    if ((rc = ws_need(ws, ws->bin_m, 4ull * plan.nb * T))) return rc;
    if ((rc = ws_need(ws, ws->bin_blk, 16ull * plan.nb))) return rc;
    if ((rc = ws_need(ws, ws->ctr, sizeof(Counters)))) return rc;
    if ((rc = ws_need(ws, ws->items, 4ull * T))) return rc;
    if ((rc = ws_need(ws, ws->item_start, 4ull * (T + 1)))) return rc;
    uint32_t* tile_start = ws->tile_start.as<uint32_t>();
    uint32_t* scan_tmp = ws->scan_tmp.as<uint32_t>();
    HIP_TRY(ctx, hipEventRecord(ws->ev[0], st), "hipEventRecord");
    HIP_TRY(ctx, launch_fill_u32(ws->ctr.as<uint32_t>(), 0u, sizeof(Counters) / 4, st), "fill");
    if (hier && tess && tess->split)
        HIP_TRY(ctx, launch_project_split_mixed(*hier, sel, tess->rows, lv.nseg, tess->cnt, cc, ws->seg.as<SegRec>(),
                                                ws->shade.as<ShadeRec>(), st),
                "k_project_split_mixed");
    else if (hier)
        HIP_TRY(ctx, launch_project_mixed(*hier, sel, lv.nseg, cc, ws->seg.as<SegRec>(), ws->shade.as<ShadeRec>(), st),
                "k_project_mixed");
    else if (dom)
        HIP_TRY(ctx, launch_project_light(lv, dom->rows, dom->grid, ws->seg.as<SegRec>(), st), "k_project_light");
    else if (tess && tess->split)
        HIP_TRY(ctx, launch_project_split(tess->base, tess->rows, lv.nseg, tess->cnt, cc, ws->seg.as<SegRec>(),
                                          ws->shade.as<ShadeRec>(), st),
                "k_project_split");
    else if (tess)
        HIP_TRY(ctx, launch_project_tess(tess->base, tess->rows, lv.nseg, tess->cnt, cc, ws->seg.as<SegRec>(),
                                         ws->shade.as<ShadeRec>(), st),
                "k_project_tess");
    else
        HIP_TRY(ctx, launch_project(lv, cc, ws->seg.as<SegRec>(), ws->shade.as<ShadeRec>(), st), "k_project");
    HIP_TRY(ctx, launch_bins(ws->seg.as<SegRec>(), lv.nseg, cc, plan, ws->bin_m.as<uint32_t>(), ws->bin_blk.as<uint4>(),
                             ws->tile_cnt.as<uint32_t>(), tile_start, ws->ctr.as<Counters>(), scan_tmp, st),
            "k_bin_count");
    // frames of up to 2^16 tiles scan and check their sizes in single-block kernels
    const bool fused = T <= kScanOneBlockTiles;
    const uint32_t kNoCap = 0xFFFFFFFFu;   // cold frames size their buffers from the sizes read back
    if (fused) {
        HIP_TRY(ctx, launch_items_scan(tile_start, T, ws->item_start.as<uint32_t>(), ws->ctr.as<Counters>(),
                                       warm ? ws->caps.pairs : kNoCap, warm ? ws->caps.items : kNoCap, st),
                "k_items_scan");
    } else {
        HIP_TRY(ctx, launch_tile_items(tile_start, T, ws->items.as<uint32_t>(), st), "k_tile_items");
        HIP_TRY(ctx, launch_exscan(ws->items.as<uint32_t>(), ws->item_start.as<uint32_t>(), T, scan_tmp, st), "k_scan");
    }
    FrameCaps caps = ws->caps;
    uint32_t pairs = 0, n_items = 0;
    if (!warm) {
        uint32_t sizes1[2] = {0, 0};
        HIP_TRY(ctx, hipMemcpyAsync(&sizes1[0], tile_start + T, 4, hipMemcpyDeviceToHost, st), "copy");
        HIP_TRY(ctx, hipMemcpyAsync(&sizes1[1], ws->item_start.as<uint32_t>() + T, 4, hipMemcpyDeviceToHost, st),
                "copy");
        HIP_TRY(ctx, hipStreamSynchronize(st), "sync");
        pairs = sizes1[0];
        n_items = sizes1[1];
        ws->last_nseg = lv.nseg;
        ws->last_ntiles = T;
        ws->last_pairs = pairs;
        out->pairs = pairs;
        if (!tiles_too) {
            HIP_TRY(ctx, hipMemcpy(&out->ctr, ws->ctr.p, sizeof(Counters), hipMemcpyDeviceToHost), "copy");
            return HAIR_OK;
        }
        caps.pairs = std::max(caps.pairs, cap_of(pairs));
        caps.items = std::max(caps.items, cap_of(n_items));
    }
    if ((rc = ws_need(ws, ws->list, 4ull * caps.pairs))) return rc;
    if ((rc = ws_need(ws, ws->item_base, 4ull * kTilePix * caps.items))) return rc;
    if ((rc = ws_need(ws, ws->item_tab, 8ull * caps.items))) return rc;
    for (DevBuf* b : {&ws->pix_cnt, &ws->pix_kmin, &ws->pix_kmax, &ws->pix_off})
        if ((rc = ws_need(ws, *b, 4 * TP))) return rc;
    if (lv.kind == 2 && (rc = ws_need(ws, ws->pix_thick, TP))) return rc;
    for (DevBuf* b : {&ws->tile_tot, &ws->tile_nb})
        if ((rc = ws_need(ws, *b, 4ull * T))) return rc;
    if ((rc = ws_need(ws, ws->batch_mask, 4ull * T * (kTilePix / 32)))) return rc;
    for (DevBuf* b : {&ws->frag_base, &ws->batch_start})
        if ((rc = ws_need(ws, *b, 4ull * (T + 1)))) return rc;
    FrameBufs f;
    memset(&f, 0, sizeof(f));
    f.T = T;
    f.ntx = ntx;
    f.seg = ws->seg.as<SegRec>();
    f.shade = ws->shade.as<ShadeRec>();
    f.tile_start = tile_start;
    f.list = ws->list.as<uint32_t>();
    f.item_start = ws->item_start.as<uint32_t>();
    f.item_tab = ws->item_tab.as<uint2>();
    f.item_base = ws->item_base.as<uint32_t>();
    f.pix_cnt = ws->pix_cnt.as<uint32_t>();
    f.pix_kmin = ws->pix_kmin.as<uint32_t>();
    f.pix_kmax = ws->pix_kmax.as<uint32_t>();
    f.pix_off = ws->pix_off.as<uint32_t>();
    f.pix_thick = lv.kind == 2 ? ws->pix_thick.as<uint8_t>() : nullptr;
    f.tile_tot = ws->tile_tot.as<uint32_t>();
    f.tile_nb = ws->tile_nb.as<uint32_t>();
    f.batch_mask = ws->batch_mask.as<uint32_t>();
    f.frag_base = ws->frag_base.as<uint32_t>();
    f.batch_start = ws->batch_start.as<uint32_t>();
    f.ctr = ws->ctr.as<Counters>();
    // (the backward pass accumulates per list entry, so its records keep list indices)
    f.gid = grad == nullptr && lv.nseg < (1 << 24);
    if (!fused) HIP_TRY(ctx, launch_check_caps(f, caps, 1, st), "k_check_caps");
    HIP_TRY(ctx, launch_scatter(f.seg, lv.nseg, cc, plan, tile_start, ws->bin_m.as<uint32_t>(), ws->list.as<uint32_t>(),
                                f.ctr, st),
            "k_scatter");
    // (a static-scratch frame clears the image only once every buffer has been carved, so that
    // a frame too large for the scratch fails with the caller's image untouched)
    HIP_TRY(ctx, launch_fill_pix(f.pix_cnt, f.pix_kmin, f.pix_kmax, f.pix_thick, TP, ws->arena ? nullptr : rgba,
                                 (size_t)cam->width * cam->height, f.item_start, T, ws->item_tab.as<uint2>(),
                                 caps.items, st),
            "fill");
    const uint32_t item_grid = warm ? caps.items : n_items;
    HIP_TRY(ctx, launch_count(f, cc, item_grid, st), "k_count");
    HIP_TRY(ctx, launch_tile_prep(f, st), "k_tile_prep");
    if (fused) {
        HIP_TRY(ctx, launch_tile_scans(f, ws->frag_base.as<uint32_t>(), ws->batch_start.as<uint32_t>(),
                                       warm ? caps.frags : kNoCap, warm ? caps.batches : kNoCap, st),
                "k_tile_scans");
    } else {
        HIP_TRY(ctx, launch_exscan(f.tile_tot, ws->frag_base.as<uint32_t>(), T, scan_tmp, st), "k_scan");
        HIP_TRY(ctx, launch_exscan(f.tile_nb, ws->batch_start.as<uint32_t>(), T, scan_tmp, st), "k_scan");
    }
    uint32_t n_frags = 0, n_batches = 0;
    if (!warm) {
        uint32_t sizes2[2] = {0, 0};
        HIP_TRY(ctx, hipMemcpyAsync(&sizes2[0], ws->frag_base.as<uint32_t>() + T, 4, hipMemcpyDeviceToHost, st),
                "copy");
        HIP_TRY(ctx, hipMemcpyAsync(&sizes2[1], ws->batch_start.as<uint32_t>() + T, 4, hipMemcpyDeviceToHost, st),
                "copy");
        HIP_TRY(ctx, hipStreamSynchronize(st), "sync");
        n_frags = sizes2[0];
        n_batches = sizes2[1];
        caps.frags = std::max(caps.frags, cap_of(n_frags));
        caps.batches = std::max(caps.batches, cap_of(n_batches));
    }
    if ((rc = ws_need(ws, ws->frags, 8ull * caps.frags))) return rc;
    if ((rc = ws_need(ws, ws->batches, 16ull * caps.batches))) return rc;
    if (lv.kind == 2 && (rc = ws_need(ws, ws->thick_list, 4ull * caps.batches))) return rc;
    f.frags = ws->frags.as<uint2>();
    f.batches = ws->batches.as<uint4>();
    f.thick_list = lv.kind == 2 ? ws->thick_list.as<uint32_t>() : nullptr;
    if (ws->arena && rgba)
        HIP_TRY(ctx, launch_fill_f32(rgba, 0.0f, 4ull * cam->width * cam->height, st), "fill");
    if (!fused) HIP_TRY(ctx, launch_check_caps(f, caps, 2, st), "k_check_caps");
    const uint32_t batch_grid = warm ? caps.batches : n_batches;
    // (the batch records follow the emit pass, which marks a mixed frame's thick-hair pixels)
    HIP_TRY(ctx, launch_emit(f, cc, item_grid, st), "k_emit");
    HIP_TRY(ctx, launch_batch_records(f, st), "k_batch_records");
    HIP_TRY(ctx, hipEventRecord(ws->ev[5], st), "hipEventRecord");
    LightsConst lc = lights_const(lights, n_lights);
    if (views)
        for (int i = 0; i < n_lights; ++i) lc.dom[i] = views[i];
    if (dom) {
        HIP_TRY(ctx, launch_dom_resolve(f, lv, dom->rows, dom->grid, dom->K, dom->delta, cam->width, batch_grid, dom->tex, st),
                "k_dom_resolve");
    } else if (grad) {
        HIP_TRY(ctx, launch_fill_f32(grad->d_axes, 0.0f, 2ull * (tess ? tess->base.nseg : lv.nseg), st), "fill");
        HIP_TRY(ctx, launch_fill_f32(grad->d_r, 0.0f, (size_t)lv.n_owner, st), "fill");
        HIP_TRY(ctx, launch_fill_f32(grad->d_sig, 0.0f, 3ull * lv.n_owner, st), "fill");
        HIP_TRY(ctx, launch_batches_bwd(f, lv, cc, lc, mat_const(a.mat), batch_grid, *grad, st), "k_batch_bwd");
    } else if (rgba) {
        HIP_TRY(ctx, launch_batches(f, lv, cc, lc, mat_const(a.mat), batch_grid, rgba, dbg, st), "k_batch");
    }
    HIP_TRY(ctx, hipEventRecord(ws->ev[6], st), "hipEventRecord");
    if (defer && warm) {   // no host synchronisation: the counters land in pinned memory
        if (!ws->ctr_host)
            HIP_TRY(ctx, hipHostMalloc((void**)&ws->ctr_host, sizeof(Counters), hipHostMallocDefault), "hipHostMalloc");
        HIP_TRY(ctx, hipMemcpyAsync(ws->ctr_host, ws->ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, st), "copy");
        HIP_TRY(ctx, hipEventRecord(ws->ev[1], st), "hipEventRecord");
        out->deferred = true;
        return HAIR_OK;
    }
    HIP_TRY(ctx, hipMemcpyAsync(&out->ctr, ws->ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(ctx, hipStreamSynchronize(st), "sync");
    if (out->ctr.cap_overflow) {
        if (!warm) return fail(HAIR_EDEVICE, "frame sizes exceeded the capacities read for them");
        return run_frame(ctx, ws, a, lv, cam, lights, n_lights, rgba, dbg, st, out, tiles_too, grad, hier, sel, dom, views,
                         tess, true);
    }
    ws->caps = caps;
    if ((rc = frame_result(ctx, ws, lv.nseg, T, out))) return rc;
    n_batches = out->n_batches;
#ifdef HAIR_PHASE_STATS
    fprintf(stderr, "phase cycles: count %llu emit %llu sort %llu shade %llu blend %llu load %llu deep-slicing %llu | "
            "deep fragments %llu batches %u items %u\n",
            out->ctr.phase[0], out->ctr.phase[1], out->ctr.phase[2], out->ctr.phase[3], out->ctr.phase[4], out->ctr.phase[5],
            out->ctr.phase[6], out->ctr.phase[7], n_batches, out->ctr.sizes[1]);
#endif
    return HAIR_OK;
}

// Rows of a frame that draws the long segments of a level (or of a mixed frame's rows, hier
// and sel given) as pieces, in ws->pieces with counts in ws->sel_cnt, and the pass and level
// that render them.  Synchronises st once (the row count).
int split_rows(hair_ctx* ctx, hair_ws* ws, const LevelDev& lv, const hair_camera* cam, hipStream_t st, TessPass* tp,
               LevelDev* lv_out, const HierDev* hier = nullptr, const uint32_t* sel = nullptr) {
    int rc;
    const int n = lv.nseg;
    if ((rc = ws_need(ws, ws->sel_cnt, 4ull * (n + 1))) || (rc = ws_need(ws, ws->sel_start, 4ull * (n + 1))) ||
        (rc = ws_need(ws, ws->sel_tmp, 4 * exscan_scratch_words(n))))
        return rc;
    uint32_t* cnt = ws->sel_cnt.as<uint32_t>();
    uint32_t* start = ws->sel_start.as<uint32_t>();
    if (hier)
        HIP_TRY(ctx, launch_split_mixed(*hier, sel, n, cam_const(cam), cnt, start, ws->sel_tmp.as<uint32_t>(), st),
                "k_split_count_mixed");
    else
        HIP_TRY(ctx, launch_split(lv, cam_const(cam), cnt, start, ws->sel_tmp.as<uint32_t>(), st), "k_split_count");
    uint32_t nrows = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&nrows, start + n, 4, hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(ctx, hipStreamSynchronize(st), "sync");
    if (nrows >= (1u << 26)) return fail(HAIR_ERANGE, "%u pieces: the frame has 2^26 rows or more", nrows);
    if ((rc = ws_need(ws, ws->pieces, 4ull * std::max<uint32_t>(nrows, 1)))) return rc;
    HIP_TRY(ctx, launch_split_fill(cnt, start, n, ws->pieces.as<uint32_t>(), st), "k_split_fill");
    tp->base = lv;
    tp->rows = ws->pieces.as<uint32_t>();
    tp->cnt = cnt;
    tp->split = true;
    *lv_out = lv;
    lv_out->nseg = (int32_t)nrows;
    return HAIR_OK;
}

// A frame of a level or of a mixed frame's rows (hier and sel) — rendered, shadowed with
// views, differentiated with grad, or dumped with dbg — drawn again with its long segments
// as pieces when the first pass found any (those are culled there).  *nseg_out: the rows of
// the frame that counts.
int level_frame(hair_ctx* ctx, hair_ws* ws, const Asset& a, const LevelDev& lv, const hair_camera* cam,
                const hair_light* lights, int n_lights, float* rgba, const DebugDump* dbg, hipStream_t st,
                FrameOut* fo, GradOut* grad = nullptr, const DomView* views = nullptr, uint32_t* nseg_out = nullptr,
                const HierDev* hier = nullptr, const uint32_t* sel = nullptr) {
    int rc;
    if ((rc = run_frame(ctx, ws, a, lv, cam, lights, n_lights, rgba, dbg, st, fo, true, grad, hier, sel, nullptr,
                        views)))
        return rc;
    if (nseg_out) *nseg_out = (uint32_t)lv.nseg;
    if (!fo->ctr.split_needed || ws->arena) return HAIR_OK;
    TessPass tp;
    LevelDev lv2;
    if ((rc = split_rows(ctx, ws, lv, cam, st, &tp, &lv2, hier, sel))) return rc;
    if (grad) grad->rows = tp.rows;
    if (nseg_out) *nseg_out = (uint32_t)lv2.nseg;
    float first[4];
    std::copy(fo->ms, fo->ms + 4, first);
    if ((rc = run_frame(ctx, ws, a, lv2, cam, lights, n_lights, rgba, dbg, st, fo, true, grad, hier, sel, nullptr,
                        views, &tp)))
        return rc;
    for (int i = 0; i < 4; ++i) fo->ms[i] += first[i];   // both passes count
    return HAIR_OK;
}

}  // namespace

// =======================================================================================
extern "C" {

int hair_version(void) { return 103; }

const char* hair_last_error(void) { return g_err.c_str(); }

int hair_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

int hair_ctx_create(int32_t device, uint64_t hbm_budget_bytes, hair_ctx** out) {
    if (!out) return fail(HAIR_EINVAL, "null output pointer");
    *out = nullptr;
    auto ctx = std::make_unique<hair_ctx>();
    ctx->device = device;
    if (device < -1) return fail(HAIR_EINVAL, "device %d", device);
    if (device >= 0) {
        const int n = hair_device_count();
        if (device >= n) return fail(HAIR_EDEVICE, "device %d not present (%d devices)", device, n);
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) return fail(HAIR_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
        size_t free_b = 0, total_b = 0;
        e = hipMemGetInfo(&free_b, &total_b);
        if (e != hipSuccess) return fail(HAIR_EDEVICE, "hipMemGetInfo: %s", hipGetErrorString(e));
        ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)total_b);
        // set-up of hair_render_noalloc: the device's scratch address and a workspace over it
        // whose timing events exist before any frame, so that its frames create nothing
        unsigned char* sp = nullptr;
        e = scratch_ptr(device, &sp);
        if (e != hipSuccess) return fail(HAIR_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        hair_ws* fw = new hair_ws();
        fw->ctx = ctx.get();
        fw->arena = sp;
        fw->arena_bytes = kScratchBytes;
        ctx->fixed_ws = fw;
        int rc = ws_events(fw);
        if (rc) {
            hair_ws_destroy(fw);
            ctx->fixed_ws = nullptr;
            return rc;
        }
    } else {
        ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (1ull << 40);
    }
    *out = ctx.release();
    return HAIR_OK;
}

int hair_ctx_destroy(hair_ctx* ctx) {
    if (!ctx) return fail(HAIR_EINVAL, "null context");
    if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
    for (auto& kv : ctx->assets) free_asset(ctx, kv.second);
    if (ctx->default_ws) hair_ws_destroy(ctx->default_ws);
    if (ctx->fixed_ws) hair_ws_destroy(ctx->fixed_ws);
    delete ctx;
    return HAIR_OK;
}

int hair_ctx_memory(hair_ctx* ctx, uint64_t* used, uint64_t* budget) {
    if (!ctx) return fail(HAIR_EINVAL, "null context");
    std::lock_guard<std::mutex> g(ctx->mu);
    if (used) *used = ctx->used;
    if (budget) *budget = ctx->budget;
    return HAIR_OK;
}

int hair_ws_create(hair_ctx* ctx, uint64_t max_bytes, hair_ws** out) {
    int rc;
    if (!out) return fail(HAIR_EINVAL, "null output pointer");
    *out = nullptr;
    if ((rc = check_ctx(ctx))) return rc;
    hair_ws* ws = new hair_ws();
    ws->ctx = ctx;
    ws->max_bytes = max_bytes;
    *out = ws;
    return HAIR_OK;
}

int hair_ws_destroy(hair_ws* ws) {
    if (!ws) return fail(HAIR_EINVAL, "null workspace");
    hair_ctx* ctx = ws->ctx;
    if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
    // a frame of hair_render_async still reads and writes the buffers: let it end first
    if (ws->pending.active && !ws->pending.done && ws->events) (void)hipEventSynchronize(ws->ev[1]);
    ws->pending.active = false;
    if (!ws->arena)
        for (DevBuf* b : ws_buffers(ws)) ctx_free(ctx, *b, ws);
    if (ws->ctr_host) (void)hipHostFree(ws->ctr_host);
    if (ws->events)
        for (auto& e : ws->ev) (void)hipEventDestroy(e);
    if (ctx->default_ws == ws) ctx->default_ws = nullptr;
    delete ws;
    return HAIR_OK;
}

int hair_ws_memory(hair_ws* ws, uint64_t* held_bytes, uint64_t* max_bytes) {
    if (!ws) return fail(HAIR_EINVAL, "null workspace");
    std::lock_guard<std::mutex> g(ws->mu);
    if (held_bytes) *held_bytes = ws->arena ? 0 : ws->held;
    if (max_bytes) *max_bytes = ws->max_bytes;
    return HAIR_OK;
}

int hair_ws_set_limit(hair_ws* ws, uint64_t max_bytes) {
    if (!ws) return fail(HAIR_EINVAL, "null workspace");
    std::lock_guard<std::mutex> g(ws->mu);
    ws->max_bytes = max_bytes;
    return HAIR_OK;
}

int hair_ws_trim(hair_ws* ws) {
    if (!ws) return fail(HAIR_EINVAL, "null workspace");
    hair_ctx* ctx = ws->ctx;
    std::lock_guard<std::mutex> g(ws->mu);
    if (ws->pending.active)
        return fail(HAIR_EINVAL, "the workspace holds a frame of hair_render_async: call hair_ws_finish first");
    if (ws->arena) return HAIR_OK;
    if (ctx->device >= 0) HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    for (DevBuf* b : ws_buffers(ws)) ctx_free(ctx, *b, ws);
    ws->caps = FrameCaps{};
    ws->dom_n = 0;
    return HAIR_OK;
}

uint64_t hair_ws_estimate(int64_t n_segments, int32_t width, int32_t height, int64_t pairs_estimate) {
    if (n_segments < 0) n_segments = 0;
    if (width < 1) width = 1;
    if (height < 1) height = 1;
    const uint64_t T = (uint64_t)((width + kTile - 1) / kTile) * (uint64_t)((height + kTile - 1) / kTile);
    if (pairs_estimate <= 0) pairs_estimate = 4 * n_segments;
    const uint64_t P = (uint64_t)pairs_estimate;
    const uint64_t items = T + P / kTilePix + 1;
    const uint64_t frags = 8 * P;   // fragments per (tile, segment) pair at strand widths ~ 4-5
    // per-block tile counts (4 B per block and tile) and statistics (16 B per block, bounded by T)
    const uint64_t bin_nb = (uint64_t)bin_plan((int32_t)std::min<int64_t>(n_segments, INT32_MAX), (int32_t)T).nb;
    const uint64_t raw = (sizeof(SegRec) + sizeof(ShadeRec)) * (uint64_t)std::max<int64_t>(n_segments, 1) +
                         4ull * (2 * T + 1) + 20ull * bin_nb * T +
                         4ull * (2 * T + 2) + 4 * P + (4ull * kTilePix + 8) * items + 1ull * T * kTilePix +
                         4ull * 4 * T * kTilePix + 4ull * 4 * (T + 1) + 32 * T + 8 * frags + 20 * (T + frags / 512) +
                         sizeof(Counters) + 4 * exscan_scratch_words(T);
    return raw + raw / 4 + 27 * 256;
}

int hair_upload(hair_ctx* ctx, int32_t n_strands, int32_t verts_per_strand, const float* xyz_soa,
                const float* width, const float* sigma_a_soa, const hair_material* material, void* stream,
                int32_t* asset_out) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!asset_out) return fail(HAIR_EINVAL, "null asset output");
    *asset_out = -1;
    if (n_strands < 1) return fail(HAIR_EINVAL, "n_strands must be >= 1");
    if (verts_per_strand < 2) return fail(HAIR_EINVAL, "verts_per_strand must be >= 2");
    const int64_t nv = (int64_t)n_strands * verts_per_strand;
    if (nv > (int64_t)INT32_MAX / 2) return fail(HAIR_EINVAL, "too many vertices (%lld)", (long long)nv);
    if (!xyz_soa || !width || !sigma_a_soa) return fail(HAIR_EINVAL, "null input array");
    if ((rc = validate_material(material))) return rc;
    if (!finite_all(xyz_soa, 3 * (size_t)nv)) return fail(HAIR_EINVAL, "vertex positions must be finite");
    for (int i = 0; i < n_strands; ++i)
        if (!(std::isfinite(width[i]) && width[i] > 0)) return fail(HAIR_EINVAL, "width[%d] must be finite and > 0", i);
    for (int64_t i = 0; i < 3ll * n_strands; ++i)
        if (!(std::isfinite(sigma_a_soa[i]) && sigma_a_soa[i] >= 0))
            return fail(HAIR_EINVAL, "sigma_a must be finite and >= 0");
    if ((rc = need_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    Asset a;
    a.n_strands = n_strands;
    a.V = verts_per_strand;
    a.S = verts_per_strand - 1;
    a.mat = *material;
    const size_t vb = 4ull * nv;
    if ((rc = ctx_alloc(ctx, a.x, vb)) || (rc = ctx_alloc(ctx, a.y, vb)) || (rc = ctx_alloc(ctx, a.z, vb)) ||
        (rc = ctx_alloc(ctx, a.width, 4ull * n_strands)) || (rc = ctx_alloc(ctx, a.sig, 12ull * n_strands))) {
        free_asset(ctx, a);
        return rc;
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(a.x.p, xyz_soa, vb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(a.y.p, xyz_soa + nv, vb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(a.z.p, xyz_soa + 2 * nv, vb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(a.width.p, width, 4ull * n_strands, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(a.sig.p, sigma_a_soa, 12ull * n_strands, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_asset(ctx, a);
        return dev_fail(ctx, e, "upload");
    }
    std::lock_guard<std::mutex> g(ctx->mu);
    const int id = ctx->next_id++;
    ctx->assets.emplace(id, std::move(a));
    *asset_out = id;
    return HAIR_OK;
}

int hair_release(hair_ctx* ctx, int32_t asset) {
    if (!ctx) return fail(HAIR_EINVAL, "null context");
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
    free_asset(ctx, it->second);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->assets.erase(it);
    return HAIR_OK;
}

int hair_lod_info(hair_ctx* ctx, int32_t asset, int32_t* n_levels, int32_t* counts, int32_t max_counts,
                  int32_t* segs_per_strand) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    const Asset& a = it->second;
    if (n_levels) *n_levels = (int32_t)a.levels.size();
    if (segs_per_strand) *segs_per_strand = a.S;
    if (counts) {
        if (max_counts >= 1) counts[0] = a.n_strands;
        for (int l = 1; l <= (int)a.levels.size() && l < max_counts; ++l) counts[l] = a.levels[l - 1].K;
    }
    return HAIR_OK;
}

static int alloc_level(hair_ctx* ctx, Level& l, int K, int S) {
    int rc;
    l.K = K;
    l.S = S;
    const size_t nv = (size_t)K * (S + 1), ns = (size_t)K * S;
    if ((rc = ctx_alloc(ctx, l.cx, 4 * nv)) || (rc = ctx_alloc(ctx, l.cy, 4 * nv)) || (rc = ctx_alloc(ctx, l.cz, 4 * nv)) ||
        (rc = ctx_alloc(ctx, l.ahat, 12 * ns)) || (rc = ctx_alloc(ctx, l.axes, 8 * ns)) ||
        (rc = ctx_alloc(ctx, l.n_total, 4ull * K)) || (rc = ctx_alloc(ctx, l.r, 4ull * K)) ||
        (rc = ctx_alloc(ctx, l.sig, 12ull * K))) {
        free_level(ctx, l);
        return rc;
    }
    return HAIR_OK;
}

// Groups and per-level owner lists when the levels are nested (each cluster's members lie in
// one cluster of the coarsest level) and few enough for mixed frames; otherwise none.
int build_hierarchy(hair_ctx* ctx, Asset& a, int n_levels, const int32_t* n_clusters, const int32_t* assign,
                    hipStream_t st) {
    if (n_levels < 1 || n_levels > kMaxMixedLevels) return HAIR_OK;
    const int n = a.n_strands;
    const int G = n_clusters[n_levels - 1];
    const int32_t* top = assign + (size_t)(n_levels - 1) * n;
    // group of every owner of every level
    std::vector<std::vector<int32_t>> group(n_levels + 1);
    group[0].assign(top, top + n);
    for (int l = 1; l <= n_levels; ++l) {
        const int32_t* as = assign + (size_t)(l - 1) * n;
        group[l].assign(n_clusters[l - 1], -1);
        for (int s = 0; s < n; ++s) {
            int32_t& g = group[l][as[s]];
            if (g < 0) g = top[s];
            else if (g != top[s]) return HAIR_OK;   // not nested
        }
    }
    Hierarchy h;
    h.G = G;
    h.grp_start.resize(n_levels + 1);
    h.grp_owner.resize(n_levels + 1);
    int rc = HAIR_OK;
    for (int l = 0; l <= n_levels && rc == HAIR_OK; ++l) {
        const std::vector<int32_t>& gr = group[l];
        std::vector<int32_t> start(G + 1, 0), owner(gr.size());
        for (int32_t g : gr) start[g + 1]++;
        for (int g = 0; g < G; ++g) start[g + 1] += start[g];
        std::vector<int32_t> cur(start.begin(), start.end() - 1);
        for (size_t o = 0; o < gr.size(); ++o) owner[cur[gr[o]]++] = (int32_t)o;
        if ((rc = ctx_alloc(ctx, h.grp_start[l], 4ull * (G + 1))) ||
            (rc = ctx_alloc(ctx, h.grp_owner[l], 4ull * std::max<size_t>(owner.size(), 1))))
            break;
        hipError_t e = hipMemcpyAsync(h.grp_start[l].p, start.data(), 4ull * (G + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h.grp_owner[l].p, owner.data(), 4ull * owner.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = dev_fail(ctx, e, "build_lod hierarchy");
    }
    if (rc != HAIR_OK) {
        free_hierarchy(ctx, h);
        return rc;
    }
    h.nested = true;
    a.hier = std::move(h);
    return HAIR_OK;
}

int hair_build_lod(hair_ctx* ctx, int32_t asset, int32_t n_levels, const int32_t* n_clusters, const int32_t* assign,
                   void* stream) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    Asset& a = it->second;
    if (n_levels < 0 || n_levels > 64) return fail(HAIR_EINVAL, "n_levels %d outside [0, 64]", n_levels);
    if (n_levels > 0 && (!n_clusters || !assign)) return fail(HAIR_EINVAL, "null cluster arrays");
    const int n = a.n_strands;
    std::vector<std::vector<int32_t>> members(n_levels), mstart(n_levels);
    for (int l = 0; l < n_levels; ++l) {
        const int K = n_clusters[l];
        if (K < 1 || K > n) return fail(HAIR_EINVAL, "level %d: n_clusters %d outside [1, %d]", l + 1, K, n);
        const int32_t* as = assign + (size_t)l * n;
        std::vector<int32_t> cnt(K + 1, 0);
        for (int s = 0; s < n; ++s) {
            if (as[s] < 0 || as[s] >= K) return fail(HAIR_EINVAL, "level %d: assign[%d] = %d outside [0, %d)", l + 1, s, as[s], K);
            cnt[as[s] + 1]++;
        }
        for (int c = 0; c < K; ++c)
            if (cnt[c + 1] == 0) return fail(HAIR_EINVAL, "level %d: cluster %d is empty", l + 1, c);
        for (int c = 0; c < K; ++c) cnt[c + 1] += cnt[c];
        mstart[l] = cnt;
        members[l].resize(n);
        std::vector<int32_t> cur(cnt.begin(), cnt.end() - 1);
        for (int s = 0; s < n; ++s) members[l][cur[as[s]]++] = s;   // ascending strand order per cluster
    }
    if ((rc = need_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::vector<Level> built(n_levels);
    for (int l = 0; l < n_levels; ++l) {
        const int K = n_clusters[l];
        DevBuf dm, ds;
        if ((rc = alloc_level(ctx, built[l], K, a.S)) || (rc = ctx_alloc(ctx, dm, 4ull * n)) ||
            (rc = ctx_alloc(ctx, ds, 4ull * (K + 1)))) {
            ctx_free(ctx, dm);
            for (Level& b : built) free_level(ctx, b);
            return rc;
        }
        hipError_t e = hipMemcpyAsync(dm.p, members[l].data(), 4ull * n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(ds.p, mstart[l].data(), 4ull * (K + 1), hipMemcpyHostToDevice, st);
        Level& L = built[l];
        if (e == hipSuccess)
            e = launch_build_centers(a.x.as<float>(), a.y.as<float>(), a.z.as<float>(), a.width.as<float>(),
                                     a.sig.as<float>(), n, a.V, dm.as<int32_t>(), ds.as<int32_t>(), K, L.cx.as<float>(),
                                     L.cy.as<float>(), L.cz.as<float>(), L.r.as<float>(), L.sig.as<float>(),
                                     L.n_total.as<int32_t>(), st);
        if (e == hipSuccess)
            e = launch_build_ellipses(a.x.as<float>(), a.y.as<float>(), a.z.as<float>(), a.V, dm.as<int32_t>(),
                                      ds.as<int32_t>(), K, L.cx.as<float>(), L.cy.as<float>(), L.cz.as<float>(),
                                      L.r.as<float>(), L.ahat.as<float>(), L.axes.as<float>(), st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        ctx_free(ctx, dm);
        ctx_free(ctx, ds);
        if (e != hipSuccess) {
            for (Level& b : built) free_level(ctx, b);
            return dev_fail(ctx, e, "build_lod");
        }
    }
    for (Level& old : a.levels) free_level(ctx, old);
    a.levels = std::move(built);
    free_hierarchy(ctx, a.hier);
    return build_hierarchy(ctx, a, n_levels, n_clusters, assign, st);
}

int hair_get_lod(hair_ctx* ctx, int32_t asset, int32_t level, int32_t n_clusters, float* centers, float* ahat,
                 float* axes, int32_t* n_total, float* sigma_a, float* r) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    Asset& a = it->second;
    if (level < 1 || level > (int)a.levels.size()) return fail(HAIR_ENOENT, "asset %d has no level %d", asset, level);
    Level& L = a.levels[level - 1];
    if (n_clusters != L.K) return fail(HAIR_EINVAL, "level %d has %d clusters, caller passed %d", level, L.K, n_clusters);
    if (!centers || !ahat || !axes || !n_total || !sigma_a || !r) return fail(HAIR_EINVAL, "null output array");
    if ((rc = need_device(ctx))) return rc;
    const size_t K = L.K, S = L.S, V = S + 1;
    std::vector<float> x(K * V), y(K * V), z(K * V), ah(3 * K * S);
    hipError_t e = hipMemcpy(x.data(), L.cx.p, 4 * K * V, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(y.data(), L.cy.p, 4 * K * V, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(z.data(), L.cz.p, 4 * K * V, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ah.data(), L.ahat.p, 12 * K * S, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(axes, L.axes.p, 8 * K * S, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(n_total, L.n_total.p, 4 * K, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(sigma_a, L.sig.p, 12 * K, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(r, L.r.p, 4 * K, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail(ctx, e, "get_lod");
    for (size_t i = 0; i < K * V; ++i) {
        centers[3 * i] = x[i];
        centers[3 * i + 1] = y[i];
        centers[3 * i + 2] = z[i];
    }
    const size_t ns = K * S;
    for (size_t i = 0; i < ns; ++i) {
        ahat[3 * i] = ah[i];
        ahat[3 * i + 1] = ah[ns + i];
        ahat[3 * i + 2] = ah[2 * ns + i];
    }
    return HAIR_OK;
}

int hair_set_lod(hair_ctx* ctx, int32_t asset, int32_t level, int32_t n_clusters, const float* centers,
                 const float* ahat, const float* axes, const int32_t* n_total, const float* sigma_a, const float* r,
                 void* stream) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    Asset& a = it->second;
    if (level < 1 || level > (int)a.levels.size() + 1) return fail(HAIR_ENOENT, "level %d cannot be set", level);
    if (n_clusters < 1) return fail(HAIR_EINVAL, "n_clusters must be >= 1");
    if (!centers || !ahat || !axes || !n_total || !sigma_a || !r) return fail(HAIR_EINVAL, "null input array");
    const size_t K = n_clusters, S = a.S, V = S + 1;
    if (!finite_all(centers, 3 * K * V) || !finite_all(ahat, 3 * K * S)) return fail(HAIR_EINVAL, "non-finite geometry");
    for (size_t i = 0; i < 2 * K * S; ++i)
        if (!(std::isfinite(axes[i]) && axes[i] > 0)) return fail(HAIR_EINVAL, "axes must be finite and > 0");
    for (size_t c = 0; c < K; ++c) {
        if (n_total[c] < 1) return fail(HAIR_EINVAL, "n_total must be >= 1");
        if (!(std::isfinite(r[c]) && r[c] > 0)) return fail(HAIR_EINVAL, "r must be finite and > 0");
    }
    for (size_t i = 0; i < 3 * K; ++i)
        if (!(std::isfinite(sigma_a[i]) && sigma_a[i] >= 0)) return fail(HAIR_EINVAL, "sigma_a must be finite and >= 0");
    if ((rc = need_device(ctx))) return rc;
    Level L;
    if ((rc = alloc_level(ctx, L, (int)K, (int)S))) return rc;
    std::vector<float> x(K * V), y(K * V), z(K * V), ah(3 * K * S);
    for (size_t i = 0; i < K * V; ++i) {
        x[i] = centers[3 * i];
        y[i] = centers[3 * i + 1];
        z[i] = centers[3 * i + 2];
    }
    const size_t ns = K * S;
    for (size_t i = 0; i < ns; ++i) {
        ah[i] = ahat[3 * i];
        ah[ns + i] = ahat[3 * i + 1];
        ah[2 * ns + i] = ahat[3 * i + 2];
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(L.cx.p, x.data(), 4 * K * V, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.cy.p, y.data(), 4 * K * V, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.cz.p, z.data(), 4 * K * V, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.ahat.p, ah.data(), 12 * ns, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.axes.p, axes, 8 * ns, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.n_total.p, n_total, 4 * K, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.sig.p, sigma_a, 12 * K, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(L.r.p, r, 4 * K, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_level(ctx, L);
        return dev_fail(ctx, e, "set_lod");
    }
    // the same clusters with new data keep their memberships (the nesting of per-group LoD);
    // a new level or another cluster count makes them unknown
    const bool same_clusters = level <= (int)a.levels.size() && a.levels[level - 1].K == (int)K;
    if (level == (int)a.levels.size() + 1) {
        a.levels.push_back(std::move(L));
    } else {
        free_level(ctx, a.levels[level - 1]);
        a.levels[level - 1] = std::move(L);
    }
    if (!same_clusters) free_hierarchy(ctx, a.hier);
    return HAIR_OK;
}

int hair_set_cluster_params(hair_ctx* ctx, int32_t asset, int32_t level, const float* axes, const float* r,
                            const float* sigma_a, void* stream) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    Asset& a = it->second;
    if (level < 1 || level > (int)a.levels.size()) return fail(HAIR_ENOENT, "asset %d has no level %d", asset, level);
    if ((rc = need_device(ctx))) return rc;
    Level& L = a.levels[level - 1];
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (axes) e = hipMemcpyAsync(L.axes.p, axes, 8ull * L.K * L.S, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && r) e = hipMemcpyAsync(L.r.p, r, 4ull * L.K, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && sigma_a) e = hipMemcpyAsync(L.sig.p, sigma_a, 12ull * L.K, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "set_cluster_params");
    return HAIR_OK;
}

int hair_select_level(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam, float eps_w_px, void* stream,
                      int32_t* level_out) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!level_out) return fail(HAIR_EINVAL, "null level output");
    if ((rc = validate_camera(cam))) return rc;
    if (!(std::isfinite(eps_w_px) && eps_w_px >= 0)) return fail(HAIR_EINVAL, "eps_w must be finite and >= 0");
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    if ((rc = need_device(ctx))) return rc;
    ws = ws_or_default(ctx, ws);
    std::lock_guard<std::mutex> g(ws->mu);
    const Asset& a = it->second;
    for (int l = (int)a.levels.size(); l >= 1; --l) {
        Asset* ap;
        LevelDev lv;
        if ((rc = find_level(ctx, asset, l, &ap, &lv))) return rc;
        FrameOut fo;
        if ((rc = run_frame(ctx, ws, a, lv, cam, nullptr, 0, nullptr, nullptr, (hipStream_t)stream, &fo, false)))
            return rc;
        float max_hw;
        memcpy(&max_hw, &fo.ctr.max_hw_bits, 4);
        if (fo.ctr.visible == 0 || 2.0f * max_hw <= eps_w_px) {
            *level_out = l;
            return HAIR_OK;
        }
    }
    *level_out = 0;
    return HAIR_OK;
}

static void fill_stats(hair_stats* stats, const FrameOut& fo, uint32_t nseg) {
    stats->fragments = fo.ctr.fragments;
    stats->pairs = fo.pairs;
    stats->segments = nseg;
    stats->segments_visible = fo.ctr.visible;
    stats->segments_culled_long = fo.ctr.culled_long;
    stats->overflow_pixels = fo.ctr.overflow_pixels;
    stats->ms_total = fo.ms[0];
    stats->ms_project = fo.ms[1];
    stats->ms_bin = fo.ms[2];
    stats->ms_tile = fo.ms[3];
    stats->deep_pixels = fo.ctr.deep_pixels;
    stats->batches = fo.n_batches;
}

int hair_render(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                const hair_light* lights, int32_t n_lights, float* rgba_out, void* stream, hair_stats* stats) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = validate_camera(cam))) return rc;
    if ((rc = validate_lights(lights, n_lights))) return rc;
    if (!rgba_out) return fail(HAIR_EINVAL, "null output image");
    Asset* a;
    LevelDev lv;
    if ((rc = find_level(ctx, asset, level, &a, &lv))) return rc;
    if ((rc = need_device(ctx))) return rc;
    ws = ws_or_default(ctx, ws);
    std::lock_guard<std::mutex> g(ws->mu);
    FrameOut fo;
    uint32_t nrows = 0;
    if ((rc = level_frame(ctx, ws, *a, lv, cam, lights, n_lights, rgba_out, nullptr, (hipStream_t)stream, &fo, nullptr,
                          nullptr, &nrows)))
        return rc;
    if (stats) fill_stats(stats, fo, nrows);
    if (fo.ctr.list_overflow) return fail(HAIR_ERANGE, "%u tiles hold more than 2^24 segments", fo.ctr.list_overflow);
    if (fo.ctr.overflow_pixels)
        return fail(HAIR_ERANGE, "%u pixels hold more than %d fragments at one depth key (left transparent)",
                    fo.ctr.overflow_pixels, kCap);
    return HAIR_OK;
}

int hair_render_noalloc(hair_ctx* ctx, int32_t asset, int32_t level, const hair_camera* cam, const hair_light* lights,
                        int32_t n_lights, float* rgba_out, void* stream, hair_stats* stats) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = validate_camera(cam))) return rc;
    if ((rc = validate_lights(lights, n_lights))) return rc;
    if (!rgba_out) return fail(HAIR_EINVAL, "null output image");
    Asset* a;
    LevelDev lv;
    if ((rc = find_level(ctx, asset, level, &a, &lv))) return rc;
    if ((rc = need_device(ctx))) return rc;
    hair_ws* ws = ctx->fixed_ws;
    if (!ws) return fail(HAIR_EDEVICE, "the context has no static scratch");
    std::lock_guard<std::mutex> g(ws->mu);
    FrameOut fo;
    if ((rc = run_frame(ctx, ws, *a, lv, cam, lights, n_lights, rgba_out, nullptr, (hipStream_t)stream, &fo, true,
                        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, true))) {
        // a frame rejected after its first kernels were enqueued: they end before the scratch
        // serves another call (which may come on another stream)
        if (rc == HAIR_ENOMEM) (void)hipStreamSynchronize((hipStream_t)stream);
        return rc;
    }
    if (stats) fill_stats(stats, fo, (uint32_t)lv.nseg);
    if (fo.ctr.list_overflow) return fail(HAIR_ERANGE, "%u tiles hold more than 2^24 segments", fo.ctr.list_overflow);
    if (fo.ctr.overflow_pixels)
        return fail(HAIR_ERANGE, "%u pixels hold more than %d fragments at one depth key (left transparent)",
                    fo.ctr.overflow_pixels, kCap);
    return HAIR_OK;
}

uint64_t hair_noalloc_scratch_bytes(void) { return kScratchBytes; }

int hair_render_async(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                      const hair_light* lights, int32_t n_lights, float* rgba_out, void* stream) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!ws) return fail(HAIR_EINVAL, "hair_render_async needs a workspace of its own");
    if (ws->ctx != ctx) return fail(HAIR_EINVAL, "the workspace belongs to another context");
    if ((rc = validate_camera(cam))) return rc;
    if ((rc = validate_lights(lights, n_lights))) return rc;
    if (!rgba_out) return fail(HAIR_EINVAL, "null output image");
    Asset* a;
    LevelDev lv;
    if ((rc = find_level(ctx, asset, level, &a, &lv))) return rc;
    if ((rc = need_device(ctx))) return rc;
    std::lock_guard<std::mutex> g(ws->mu);
    FrameOut fo;
    if ((rc = run_frame(ctx, ws, *a, lv, cam, lights, n_lights, rgba_out, nullptr, (hipStream_t)stream, &fo, true,
                        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, false, true)))
        return rc;
    hair_ws::Pending& pd = ws->pending;
    pd.active = true;
    pd.done = !fo.deferred;
    pd.asset = asset;
    pd.level = level;
    pd.cam = *cam;
    pd.lights.assign(lights, lights + n_lights);
    pd.rgba = rgba_out;
    pd.st = (hipStream_t)stream;
    if (pd.done) {
        pd.ctr = fo.ctr;
        pd.pairs = fo.pairs;
        pd.n_batches = fo.n_batches;
        for (int i = 0; i < 4; ++i) pd.ms[i] = fo.ms[i];
    }
    return HAIR_OK;
}

int hair_ws_finish(hair_ws* ws, hair_stats* stats) {
    if (!ws) return fail(HAIR_EINVAL, "null workspace");
    hair_ctx* ctx = ws->ctx;
    std::lock_guard<std::mutex> g(ws->mu);
    hair_ws::Pending& pd = ws->pending;
    if (!pd.active) {
        if (stats) *stats = hair_stats{};
        return HAIR_OK;
    }
    int rc;
    FrameOut fo;
    Asset* a;
    LevelDev lv;
    const int T = ((pd.cam.width + kTile - 1) / kTile) * ((pd.cam.height + kTile - 1) / kTile);
    if (!pd.done) {   // the frame's work ends before anything else happens to the workspace
        if (ctx->device >= 0) HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        HIP_TRY(ctx, hipEventSynchronize(ws->ev[1]), "hipEventSynchronize");
    }
    if ((rc = find_level(ctx, pd.asset, pd.level, &a, &lv))) {   // (released since: no rerun possible)
        pd.active = false;
        return rc;
    }
    if (pd.done) {
        fo.ctr = pd.ctr;
        fo.pairs = pd.pairs;
        fo.n_batches = pd.n_batches;
        for (int i = 0; i < 4; ++i) fo.ms[i] = pd.ms[i];
    } else {
        fo.ctr = *ws->ctr_host;
        if (fo.ctr.cap_overflow) {   // the frame outgrew the capacities: render it again, cold
            const hair_ws::Pending p = pd;
            pd.active = false;
            if ((rc = run_frame(ctx, ws, *a, lv, &p.cam, p.lights.data(), (int)p.lights.size(), p.rgba, nullptr, p.st,
                                &fo, true, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, true)))
                return rc;
        } else if ((rc = frame_result(ctx, ws, lv.nseg, T, &fo))) {
            pd.active = false;
            return rc;
        }
    }
    pd.active = false;
    uint32_t nrows = (uint32_t)lv.nseg;
    if (fo.ctr.split_needed && !ws->arena) {   // long segments: the frame again, with pieces
        TessPass tp;
        LevelDev lv2;
        if ((rc = split_rows(ctx, ws, lv, &pd.cam, pd.st, &tp, &lv2))) return rc;
        if ((rc = run_frame(ctx, ws, *a, lv2, &pd.cam, pd.lights.data(), (int)pd.lights.size(), pd.rgba, nullptr,
                            pd.st, &fo, true, nullptr, nullptr, nullptr, nullptr, nullptr, &tp)))
            return rc;
        nrows = (uint32_t)lv2.nseg;
    }
    if (stats) fill_stats(stats, fo, nrows);
    if (fo.ctr.list_overflow) return fail(HAIR_ERANGE, "%u tiles hold more than 2^24 segments", fo.ctr.list_overflow);
    if (fo.ctr.overflow_pixels)
        return fail(HAIR_ERANGE, "%u pixels hold more than %d fragments at one depth key (left transparent)",
                    fo.ctr.overflow_pixels, kCap);
    return HAIR_OK;
}

// Light frame of a directional light (float64, stored as float32): e1 = normalize(a x omega)
// with a = y (x when |omega_y| >= 0.9), e2 = omega x e1, d = -omega.
static DomBasis dom_basis(const float* vec) {
    double w[3] = {vec[0], vec[1], vec[2]};
    const double wn = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (double& x : w) x /= wn;
    const double a[3] = {std::fabs(w[1]) < 0.9 ? 0.0 : 1.0, std::fabs(w[1]) < 0.9 ? 1.0 : 0.0, 0.0};
    double e1[3] = {a[1] * w[2] - a[2] * w[1], a[2] * w[0] - a[0] * w[2], a[0] * w[1] - a[1] * w[0]};
    const double en = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (double& x : e1) x /= en;
    const double e2[3] = {w[1] * e1[2] - w[2] * e1[1], w[2] * e1[0] - w[0] * e1[2], w[0] * e1[1] - w[1] * e1[0]};
    DomBasis b;
    for (int i = 0; i < 3; ++i) {
        b.e1[i] = (float)e1[i];
        b.e2[i] = (float)e2[i];
        b.d[i] = (float)-w[i];
        b.omega[i] = (float)w[i];
    }
    return b;
}

static int validate_shadow(const hair_shadow* shadow) {
    if (!shadow) return fail(HAIR_EINVAL, "null shadow descriptor");
    if (shadow->resolution < 16 || shadow->resolution > 4096)
        return fail(HAIR_EINVAL, "shadow resolution %d outside [16, 4096]", shadow->resolution);
    if (shadow->layers < 1 || shadow->layers > kDomMaxLayers)
        return fail(HAIR_EINVAL, "shadow layers %d outside [1, %d]", shadow->layers, kDomMaxLayers);
    if (!(std::isfinite(shadow->layer_depth) && shadow->layer_depth > 0.0f))
        return fail(HAIR_EINVAL, "shadow layer_depth must be finite and > 0");
    return HAIR_OK;
}

// One shadow pass per directional light over the level lv (or, with rows, over a mixed
// frame's rows): grid, light-view raster, per-texel resolve; fills views[] for the camera
// pass and adds the passes' GPU time to *ms.  The caller holds ws->mu.
static int shadow_passes(hair_ctx* ctx, hair_ws* ws, const Asset& a, const LevelDev& lv, const ShadeRec* rows,
                         const hair_camera* cam, const hair_light* lights, int n_lights, const hair_shadow* shadow,
                         hipStream_t st, DomView* views, float* ms) {
    int rc;
    const int R = shadow->resolution, K = shadow->layers;
    int n_dom = 0;
    for (int i = 0; i < n_lights; ++i) n_dom += lights[i].kind == 0;
    const size_t texels = (size_t)R * R;
    if ((rc = ws_need(ws, ws->dom_tex, 32 * texels * std::max(n_dom, 1)))) return rc;
    if ((rc = ws_need(ws, ws->dom_grid, sizeof(DomGrid) * HAIR_MAX_LIGHTS))) return rc;
    if ((rc = ws_need(ws, ws->dom_part, 20ull * dom_bound_blocks(lv.nseg)))) return rc;
    hair_camera lcam = *cam;   // the light view's raster size; its projection is the light's own
    lcam.width = lcam.height = R;
    memset(views, 0, sizeof(DomView) * HAIR_MAX_LIGHTS);
    int m = 0;
    for (int i = 0; i < n_lights; ++i) {
        ws->dom_light[i] = -1;
        if (lights[i].kind != 0) continue;
        DomGrid* grid = ws->dom_grid.as<DomGrid>() + m;
        float4* tex = reinterpret_cast<float4*>(ws->dom_tex.as<float>() + 8 * texels * m);
        HIP_TRY(ctx, launch_dom_grid(lv, rows, dom_basis(lights[i].vec), R, ws->dom_part.as<float>(), grid, st),
                "k_dom_grid");
        const DomPass dp{grid, K, shadow->layer_depth, tex, rows};
        FrameOut fd;
        if ((rc = run_frame(ctx, ws, a, lv, &lcam, lights, n_lights, nullptr, nullptr, st, &fd, true, nullptr,
                            nullptr, nullptr, &dp)))
            return rc;
        if (fd.ctr.list_overflow) return fail(HAIR_ERANGE, "shadow map: %u tiles hold more than 2^24 segments",
                                              fd.ctr.list_overflow);
        *ms += fd.ms[0];
        views[i] = DomView{grid, tex, K, shadow->layer_depth};
        ws->dom_light[i] = m++;
    }
    ws->dom_R = R;
    ws->dom_K = K;
    ws->dom_n = m;
    return HAIR_OK;
}

int hair_render_shadowed(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                         const hair_light* lights, int32_t n_lights, const hair_shadow* shadow, float* rgba_out,
                         void* stream, hair_stats* stats) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = validate_camera(cam))) return rc;
    if ((rc = validate_lights(lights, n_lights))) return rc;
    if (!rgba_out) return fail(HAIR_EINVAL, "null output image");
    if ((rc = validate_shadow(shadow))) return rc;
    Asset* a;
    LevelDev lv;
    if ((rc = find_level(ctx, asset, level, &a, &lv))) return rc;
    if ((rc = need_device(ctx))) return rc;
    ws = ws_or_default(ctx, ws);
    std::lock_guard<std::mutex> g(ws->mu);
    const hipStream_t st = (hipStream_t)stream;
    DomView views[HAIR_MAX_LIGHTS];
    float ms_dom = 0.0f;
    if ((rc = shadow_passes(ctx, ws, *a, lv, nullptr, cam, lights, n_lights, shadow, st, views, &ms_dom))) return rc;
    FrameOut fo;
    uint32_t nrows = 0;
    if ((rc = level_frame(ctx, ws, *a, lv, cam, lights, n_lights, rgba_out, nullptr, st, &fo, nullptr, views, &nrows)))
        return rc;
    if (stats) {
        fill_stats(stats, fo, nrows);
        stats->ms_total += ms_dom;
    }
    if (fo.ctr.list_overflow) return fail(HAIR_ERANGE, "%u tiles hold more than 2^24 segments", fo.ctr.list_overflow);
    if (fo.ctr.overflow_pixels)
        return fail(HAIR_ERANGE, "%u pixels hold more than %d fragments at one depth key (left transparent)",
                    fo.ctr.overflow_pixels, kCap);
    return HAIR_OK;
}

int hair_debug_dom(hair_ws* ws, int32_t light, float* texels, float* grid) {
    if (!ws || !texels || !grid) return fail(HAIR_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(ws->mu);
    if (light < 0 || light >= HAIR_MAX_LIGHTS || ws->dom_R == 0 || ws->dom_light[light] < 0)
        return fail(HAIR_EINVAL, "light %d has no shadow map in the last shadowed render", light);
    const int m = ws->dom_light[light];
    const size_t texels_n = (size_t)ws->dom_R * ws->dom_R;
    hipError_t e = hipMemcpy(texels, ws->dom_tex.as<float>() + 8 * texels_n * m, 32 * texels_n, hipMemcpyDeviceToHost);
    DomGrid gr;
    if (e == hipSuccess) e = hipMemcpy(&gr, ws->dom_grid.as<DomGrid>() + m, sizeof(DomGrid), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail(ws->ctx, e, "debug_dom");
    for (int i = 0; i < 3; ++i) {
        grid[i] = gr.b.e1[i];
        grid[3 + i] = gr.b.e2[i];
        grid[6 + i] = gr.b.d[i];
        grid[9 + i] = gr.b.omega[i];
    }
    grid[12] = gr.u0;
    grid[13] = gr.v0;
    grid[14] = gr.s;
    grid[15] = gr.z_ref;
    return HAIR_OK;
}

// The asset's nested hierarchy as device views (levels 0..n_levels).
static int mixed_hierarchy(hair_ctx* ctx, int32_t asset, Asset** a_out, HierDev* h) {
    auto it = ctx->assets.find(asset);
    if (it == ctx->assets.end()) return fail(HAIR_ENOENT, "unknown asset %d", asset);
    Asset& a = it->second;
    if (!a.hier.nested)
        return fail(HAIR_EINVAL, "asset %d has no nested LoD hierarchy (hair_build_lod with 1..%d levels whose "
                    "clusters each lie inside one cluster of the coarsest level)", asset, kMaxMixedLevels);
    memset(h, 0, sizeof(*h));
    h->n_levels = (int)a.levels.size();
    h->G = a.hier.G;
    h->S = a.S;
    for (int l = 0; l <= h->n_levels; ++l) {
        Asset* dummy;
        int rc = find_level(ctx, asset, l, &dummy, &h->lv[l]);
        if (rc) return rc;
        if (h->lv[l].nseg >= (1 << 28)) return fail(HAIR_ERANGE, "level %d has 2^28 segments or more", l);
        h->grp_start[l] = a.hier.grp_start[l].as<int32_t>();
        h->grp_owner[l] = a.hier.grp_owner[l].as<int32_t>();
    }
    *a_out = &a;
    return HAIR_OK;
}

int hair_lod_groups(hair_ctx* ctx, int32_t asset, int32_t* n_groups) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!n_groups) return fail(HAIR_EINVAL, "null output");
    Asset* a;
    HierDev h;
    if ((rc = mixed_hierarchy(ctx, asset, &a, &h))) return rc;
    *n_groups = h.G;
    return HAIR_OK;
}

int hair_lod_init(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam, float eps_w_px, int32_t* levels,
                  void* stream) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = validate_camera(cam))) return rc;
    if (!levels) return fail(HAIR_EINVAL, "null levels");
    if (!(std::isfinite(eps_w_px) && eps_w_px > 0)) return fail(HAIR_EINVAL, "eps_w must be finite and > 0");
    Asset* a;
    HierDev h;
    if ((rc = mixed_hierarchy(ctx, asset, &a, &h))) return rc;
    if ((rc = need_device(ctx))) return rc;
    (void)ws;
    HIP_TRY(ctx, launch_lod_init(h, cam_const(cam), eps_w_px, levels, (hipStream_t)stream), "k_lod_init");
    HIP_TRY(ctx, hipStreamSynchronize((hipStream_t)stream), "sync");
    return HAIR_OK;
}

// A mixed frame (optionally shadowed): rows of every (group, segment) at its level, then the
// shadow passes over those rows (their world data from the camera projection of the rows),
// the camera frame, and the deferred level update.
static int render_mixed(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam, const hair_light* lights,
                        int32_t n_lights, int32_t* levels, float eps_w_px, const hair_shadow* shadow, float* rgba_out,
                        void* stream, hair_stats* stats) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = validate_camera(cam))) return rc;
    if ((rc = validate_lights(lights, n_lights))) return rc;
    if (!rgba_out || !levels) return fail(HAIR_EINVAL, "null output image or levels");
    if (!std::isfinite(eps_w_px)) return fail(HAIR_EINVAL, "eps_w must be finite");
    if (shadow && (rc = validate_shadow(shadow))) return rc;
    Asset* a;
    HierDev h;
    if ((rc = mixed_hierarchy(ctx, asset, &a, &h))) return rc;
    if ((rc = need_device(ctx))) return rc;
    ws = ws_or_default(ctx, ws);
    std::lock_guard<std::mutex> g(ws->mu);
    hipStream_t st = (hipStream_t)stream;
    const int GS = h.G * h.S;
    if ((rc = ws_need(ws, ws->sel_cnt, 4ull * (GS + 1))) || (rc = ws_need(ws, ws->sel_start, 4ull * (GS + 1))) ||
        (rc = ws_need(ws, ws->sel_tmp, 4 * exscan_scratch_words(GS))))
        return rc;
    uint32_t* cnt = ws->sel_cnt.as<uint32_t>();
    HIP_TRY(ctx, launch_fill_u32(cnt + GS, 0u, 1, st), "fill");
    HIP_TRY(ctx, launch_select(h, levels, cnt, ws->sel_start.as<uint32_t>(), ws->sel_tmp.as<uint32_t>(), st),
            "k_sel_count");
    uint32_t nsel = 0, bad = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&nsel, ws->sel_start.as<uint32_t>() + GS, 4, hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(ctx, hipMemcpyAsync(&bad, cnt + GS, 4, hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(ctx, hipStreamSynchronize(st), "sync");
    if (bad) return fail(HAIR_EINVAL, "%u entries of levels lie outside [0, %d]", bad, h.n_levels);
    if ((rc = ws_need(ws, ws->sel, 4ull * std::max<uint32_t>(nsel, 1)))) return rc;
    HIP_TRY(ctx, launch_select_fill(h, levels, ws->sel_start.as<uint32_t>(), ws->sel.as<uint32_t>(), st), "k_sel_fill");
    LevelDev lv;
    memset(&lv, 0, sizeof(lv));
    lv.kind = 2;
    lv.nseg = (int32_t)nsel;
    lv.S = a->S;
    DomView views[HAIR_MAX_LIGHTS];
    float ms_dom = 0.0f;
    if (shadow) {
        // the rows' shading records (world endpoints and cross-sections) feed the shadow passes;
        // the camera frame projects them again into the same buffers
        if ((rc = ws_need(ws, ws->seg, sizeof(SegRec) * (size_t)std::max<uint32_t>(nsel, 1))) ||
            (rc = ws_need(ws, ws->shade, sizeof(ShadeRec) * (size_t)std::max<uint32_t>(nsel, 1))))
            return rc;
        HIP_TRY(ctx, launch_project_mixed(h, ws->sel.as<uint32_t>(), (int32_t)nsel, cam_const(cam),
                                          ws->seg.as<SegRec>(), ws->shade.as<ShadeRec>(), st),
                "k_project_mixed");
        if ((rc = shadow_passes(ctx, ws, *a, lv, ws->shade.as<ShadeRec>(), cam, lights, n_lights, shadow, st, views,
                                &ms_dom)))
            return rc;
    }
    FrameOut fo;
    uint32_t nrows = 0;
    if ((rc = level_frame(ctx, ws, *a, lv, cam, lights, n_lights, rgba_out, nullptr, st, &fo, nullptr,
                          shadow ? views : nullptr, &nrows, &h, ws->sel.as<uint32_t>())))
        return rc;
    if (eps_w_px > 0) {
        HIP_TRY(ctx, launch_lod_update(h, cam_const(cam), eps_w_px, levels, st), "k_lod_update");
        HIP_TRY(ctx, hipStreamSynchronize(st), "sync");
    }
    if (stats) {
        fill_stats(stats, fo, nrows);
        stats->ms_total += ms_dom;
    }
    if (fo.ctr.list_overflow) return fail(HAIR_ERANGE, "%u tiles hold more than 2^24 segments", fo.ctr.list_overflow);
    if (fo.ctr.overflow_pixels)
        return fail(HAIR_ERANGE, "%u pixels hold more than %d fragments at one depth key (left transparent)",
                    fo.ctr.overflow_pixels, kCap);
    return HAIR_OK;
}

int hair_render_mixed(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam, const hair_light* lights,
                      int32_t n_lights, int32_t* levels, float eps_w_px, float* rgba_out, void* stream,
                      hair_stats* stats) {
    return render_mixed(ctx, ws, asset, cam, lights, n_lights, levels, eps_w_px, nullptr, rgba_out, stream, stats);
}

int hair_render_mixed_shadowed(hair_ctx* ctx, hair_ws* ws, int32_t asset, const hair_camera* cam,
                               const hair_light* lights, int32_t n_lights, int32_t* levels, float eps_w_px,
                               const hair_shadow* shadow, float* rgba_out, void* stream, hair_stats* stats) {
    if (!shadow) return fail(HAIR_EINVAL, "null shadow descriptor");
    return render_mixed(ctx, ws, asset, cam, lights, n_lights, levels, eps_w_px, shadow, rgba_out, stream, stats);
}

int hair_render_curved(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                       const hair_light* lights, int32_t n_lights, int32_t max_px, int32_t max_sub, float* rgba_out,
                       void* stream, hair_stats* stats) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = validate_camera(cam))) return rc;
    if ((rc = validate_lights(lights, n_lights))) return rc;
    if (!rgba_out) return fail(HAIR_EINVAL, "null output image");
    if (level < 1) return fail(HAIR_EINVAL, "curved centre lines need a thick-hair level (>= 1)");
    if (max_px < 1 || max_px > 4096) return fail(HAIR_EINVAL, "max_px %d outside [1, 4096]", max_px);
    if (max_sub < 1 || max_sub > 16) return fail(HAIR_EINVAL, "max_sub %d outside [1, 16]", max_sub);
    Asset* a;
    LevelDev base;
    if ((rc = find_level(ctx, asset, level, &a, &base))) return rc;
    if (base.nseg >= (1 << 27)) return fail(HAIR_ERANGE, "level %d has 2^27 segments or more", level);
    if ((rc = need_device(ctx))) return rc;
    ws = ws_or_default(ctx, ws);
    std::lock_guard<std::mutex> g(ws->mu);
    const hipStream_t st = (hipStream_t)stream;
    const int n = base.nseg;
    if ((rc = ws_need(ws, ws->sel_cnt, 4ull * (n + 1))) || (rc = ws_need(ws, ws->sel_start, 4ull * (n + 1))) ||
        (rc = ws_need(ws, ws->sel_tmp, 4 * exscan_scratch_words(n))))
        return rc;
    uint32_t* cnt = ws->sel_cnt.as<uint32_t>();
    uint32_t* start = ws->sel_start.as<uint32_t>();
    HIP_TRY(ctx, launch_tess(base, cam_const(cam), max_px, max_sub, cnt, start, ws->sel_tmp.as<uint32_t>(), st),
            "k_tess_count");
    uint32_t nrows = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&nrows, start + n, 4, hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(ctx, hipStreamSynchronize(st), "sync");
    if ((rc = ws_need(ws, ws->sel, 4ull * std::max<uint32_t>(nrows, 1)))) return rc;
    HIP_TRY(ctx, launch_tess_fill(cnt, start, n, ws->sel.as<uint32_t>(), st), "k_tess_fill");
    LevelDev lv = base;
    lv.nseg = (int32_t)nrows;
    const TessPass tp{base, ws->sel.as<uint32_t>(), cnt};
    FrameOut fo;
    if ((rc = run_frame(ctx, ws, *a, lv, cam, lights, n_lights, rgba_out, nullptr, st, &fo, true, nullptr, nullptr,
                        nullptr, nullptr, nullptr, &tp)))
        return rc;
    if (stats) fill_stats(stats, fo, nrows);
    if (fo.ctr.list_overflow) return fail(HAIR_ERANGE, "%u tiles hold more than 2^24 segments", fo.ctr.list_overflow);
    if (fo.ctr.overflow_pixels)
        return fail(HAIR_ERANGE, "%u pixels hold more than %d fragments at one depth key (left transparent)",
                    fo.ctr.overflow_pixels, kCap);
    return HAIR_OK;
}

int hair_render_backward(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                         const hair_light* lights, int32_t n_lights, const float* d_rgba, float* d_axes, float* d_r,
                         float* d_sigma_a, void* stream) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = validate_camera(cam))) return rc;
    if ((rc = validate_lights(lights, n_lights))) return rc;
    if (!d_rgba || !d_axes || !d_r || !d_sigma_a) return fail(HAIR_EINVAL, "null gradient array");
    if (level < 1) return fail(HAIR_EINVAL, "the backward pass needs a thick-hair level (>= 1)");
    Asset* a;
    LevelDev lv;
    if ((rc = find_level(ctx, asset, level, &a, &lv))) return rc;
    if ((rc = need_device(ctx))) return rc;
    ws = ws_or_default(ctx, ws);
    std::lock_guard<std::mutex> g(ws->mu);
    GradOut grad{d_rgba, d_axes, d_r, d_sigma_a, nullptr};
    FrameOut fo;
    if ((rc = level_frame(ctx, ws, *a, lv, cam, lights, n_lights, nullptr, nullptr, (hipStream_t)stream, &fo, &grad)))
        return rc;
    if (fo.ctr.overflow_pixels)
        return fail(HAIR_ERANGE, "%u pixels need more than 64 slices of %d fragments (their gradient is missing)",
                    fo.ctr.overflow_pixels, kCap);
    return HAIR_OK;
}

int hair_debug_issue_rate(hair_ctx* ctx, int32_t kind, int32_t iters, double* ops_per_s) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (kind < 0 || kind > 5) return fail(HAIR_EINVAL, "probe kind %d outside [0, 5]", kind);
    if (iters < 1 || iters > (1 << 20)) return fail(HAIR_EINVAL, "iters %d outside [1, 2^20]", iters);
    if (!ops_per_s) return fail(HAIR_EINVAL, "null output pointer");
    if ((rc = need_device(ctx))) return rc;
    hair_ws* ws = ctx->fixed_ws;
    if (!ws) return fail(HAIR_EDEVICE, "the context has no static scratch");
    std::lock_guard<std::mutex> g(ws->mu);
    const int blocks = 256 * 32;                     // 32 blocks of 4 waves per CU: full occupancy
    float* out = reinterpret_cast<float*>(ws->arena);
    HIP_TRY(ctx, launch_probe_rate(kind, blocks, 1, out, nullptr), "k_probe_rate");   // warm-up
    HIP_TRY(ctx, hipEventRecord(ws->ev[0], nullptr), "hipEventRecord");
    HIP_TRY(ctx, launch_probe_rate(kind, blocks, iters, out, nullptr), "k_probe_rate");
    HIP_TRY(ctx, hipEventRecord(ws->ev[6], nullptr), "hipEventRecord");
    HIP_TRY(ctx, hipEventSynchronize(ws->ev[6]), "hipEventSynchronize");
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ws->ev[0], ws->ev[6]), "elapsed");
    *ops_per_s = (double)blocks * 256.0 * 8.0 * (double)iters / (ms * 1e-3);
    return HAIR_OK;
}

int hair_debug_segments(hair_ws* ws, int64_t n, int32_t* rec_i, float* rec_f) {
    if (!ws || !rec_i || !rec_f) return fail(HAIR_EINVAL, "null argument");
    if (n != ws->last_nseg) return fail(HAIR_EINVAL, "last render had %lld segments", (long long)ws->last_nseg);
    std::lock_guard<std::mutex> g(ws->mu);
    std::vector<SegRec> h(std::max<int64_t>(n, 1));
    hipError_t e = hipMemcpy(h.data(), ws->seg.p, sizeof(SegRec) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail(ws->ctx, e, "debug_segments");
    for (int64_t i = 0; i < n; ++i) {
        const SegRec& s = h[i];
        rec_i[6 * i + 0] = s.xa; rec_i[6 * i + 1] = s.ya; rec_i[6 * i + 2] = s.xb; rec_i[6 * i + 3] = s.yb;
        rec_i[6 * i + 4] = s.hwfx & kHwMask;
        rec_i[6 * i + 5] = ((s.hwfx & kFlagVisible) ? 1 : 0) | ((s.hwfx & kFlagNegSide) ? 2 : 0) |
                           ((s.hwfx & kFlagCulledLong) ? 4 : 0) | ((s.hwfx & kFlagThick) ? 8 : 0);
        rec_f[3 * i + 0] = s.iza; rec_f[3 * i + 1] = s.izb; rec_f[3 * i + 2] = s.hw;
    }
    return HAIR_OK;
}

int hair_debug_bins(hair_ws* ws, int64_t n_tiles, uint32_t* tile_start, int64_t n_pairs, uint32_t* tile_segs) {
    if (!ws || !tile_start || !tile_segs) return fail(HAIR_EINVAL, "null argument");
    if (n_tiles != ws->last_ntiles || n_pairs != ws->last_pairs)
        return fail(HAIR_EINVAL, "last render had %lld tiles and %lld pairs", (long long)ws->last_ntiles,
                    (long long)ws->last_pairs);
    std::lock_guard<std::mutex> g(ws->mu);
    hipError_t e = hipMemcpy(tile_start, ws->tile_start.p, 4 * (size_t)(n_tiles + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess && n_pairs) e = hipMemcpy(tile_segs, ws->list.p, 4 * n_pairs, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail(ws->ctx, e, "debug_bins");
    return HAIR_OK;
}

int hair_debug_fragments(hair_ctx* ctx, hair_ws* ws, int32_t asset, int32_t level, const hair_camera* cam,
                         const hair_light* lights, int32_t n_lights, int32_t x0, int32_t y0, int32_t w, int32_t h,
                         uint32_t* counts, int64_t cap, uint32_t* keys, uint32_t* segs, float* alpha, float* hoff,
                         void* stream) {
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = validate_camera(cam))) return rc;
    if ((rc = validate_lights(lights, n_lights))) return rc;
    if (w < 1 || h < 1 || x0 < 0 || y0 < 0 || x0 + w > cam->width || y0 + h > cam->height)
        return fail(HAIR_EINVAL, "debug rectangle outside the image");
    if (!counts || !keys || !segs || !alpha || !hoff || cap < 1) return fail(HAIR_EINVAL, "null output");
    Asset* a;
    LevelDev lv;
    if ((rc = find_level(ctx, asset, level, &a, &lv))) return rc;
    if ((rc = need_device(ctx))) return rc;
    ws = ws_or_default(ctx, ws);
    std::lock_guard<std::mutex> g(ws->mu);
    const int npx = w * h;
    // per-pixel room in the dump: a batch's worth, or an even share of cap when that is larger
    const int stride = (int)std::min<int64_t>(cap, std::max<int64_t>((int64_t)kCap, std::min<int64_t>(cap / (w * h), 1 << 24)));
    DevBuf img, dc, dk, ds, da, dh;
    const size_t ent = (size_t)npx * stride;
    auto cleanup = [&]() { for (DevBuf* b : {&img, &dc, &dk, &ds, &da, &dh}) ctx_free(ctx, *b); };
    if ((rc = ctx_alloc(ctx, img, 16ull * cam->width * cam->height)) || (rc = ctx_alloc(ctx, dc, 4ull * npx)) ||
        (rc = ctx_alloc(ctx, dk, 4 * ent)) || (rc = ctx_alloc(ctx, ds, 4 * ent)) || (rc = ctx_alloc(ctx, da, 4 * ent)) ||
        (rc = ctx_alloc(ctx, dh, 4 * ent))) {
        cleanup();
        return rc;
    }
    {
        hipError_t ef = launch_fill_u32(dc.as<uint32_t>(), 0u, (size_t)npx, (hipStream_t)stream);
        if (ef != hipSuccess) {
            cleanup();
            return dev_fail(ctx, ef, "fill");
        }
    }
    DebugDump dbg{x0, y0, w, h, stride, dc.as<uint32_t>(), dk.as<uint32_t>(), ds.as<uint32_t>(), da.as<float>(),
                  dh.as<float>()};
    FrameOut fo;
    rc = level_frame(ctx, ws, *a, lv, cam, lights, n_lights, img.as<float>(), &dbg, (hipStream_t)stream, &fo);
    if (rc) {
        cleanup();
        return rc;
    }
    std::vector<uint32_t> c(npx), k(ent), s(ent);
    std::vector<float> al(ent), ho(ent);
    hipError_t e = hipMemcpy(c.data(), dc.p, 4ull * npx, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(k.data(), dk.p, 4 * ent, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(s.data(), ds.p, 4 * ent, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(al.data(), da.p, 4 * ent, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ho.data(), dh.p, 4 * ent, hipMemcpyDeviceToHost);
    cleanup();
    if (e != hipSuccess) return dev_fail(ctx, e, "debug_fragments");
    int64_t total = 0;
    for (int i = 0; i < npx; ++i) {
        if (c[i] > (uint32_t)stride) return fail(HAIR_ERANGE, "pixel holds %u fragments, above %d", c[i], stride);
        total += c[i];
    }
    if (total > cap) return fail(HAIR_ERANGE, "%lld fragments do not fit cap %lld", (long long)total, (long long)cap);
    int64_t o = 0;
    for (int i = 0; i < npx; ++i) {
        counts[i] = c[i];
        for (uint32_t r = 0; r < c[i]; ++r, ++o) {
            const size_t src = (size_t)i * stride + r;
            keys[o] = k[src]; segs[o] = s[src]; alpha[o] = al[src]; hoff[o] = ho[src];
        }
    }
    if (fo.ctr.overflow_pixels) return fail(HAIR_ERANGE, "%u pixels exceed capacity", fo.ctr.overflow_pixels);
    (void)0;
    return HAIR_OK;
}

}  // extern "C"
