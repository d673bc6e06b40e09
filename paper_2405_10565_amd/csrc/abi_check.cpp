// abi_check: drives every entry point of the C-ABI (include/hair.h) once or more and checks
// the returned status codes, so that the host layer (argument checking, workspaces, level
// management, the frame drivers) can be run under host-side sanitizers.
//
//   abi_check --host-only   a host-only context (device -1): argument checking and error paths
//   abi_check --device N    the same on device N, then every frame path on a small synthetic
//                           asset: strands, thick-hair levels, shadows, curved and mixed
//                           frames, the backward pass, asynchronous and allocation-free frames,
//                           long segments drawn in pieces, and the debug exports
//
// Exit status 0 when every check holds; each failed check is printed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/hair.h"

namespace {

int g_fail = 0, g_checks = 0;

void expect(bool ok, const char* what, int line) {
    ++g_checks;
    if (!ok) {
        ++g_fail;
        std::fprintf(stderr, "abi_check: FAILED line %d: %s (last error: %s)\n", line, what, hair_last_error());
    }
}
#define EXPECT(cond) expect((cond), #cond, __LINE__)
#define EXPECT_RC(call, code) expect((call) == (code), #call " == " #code, __LINE__)

struct Asset {
    int n = 0, V = 0;
    std::vector<float> xyz, width, sigma;
};

// n strands of V vertices hanging in front of the camera (z in [-1.3, -0.9]); strand 0 ends in a
// segment about 1200 px long at 256 x 256 (drawn in pieces).
Asset make_asset(int n, int V) {
    Asset a;
    a.n = n;
    a.V = V;
    a.xyz.assign(3ull * n * V, 0.0f);
    a.width.assign(n, 80e-6f);
    a.sigma.assign(3ull * n, 0.0f);
    unsigned s = 12345u;
    auto rnd = [&]() { s = s * 1664525u + 1013904223u; return (s >> 8) * (1.0f / 16777216.0f); };
    for (int i = 0; i < n; ++i) {
        const float x0 = -0.25f + 0.5f * rnd(), z0 = -0.9f - 0.4f * rnd(), ph = 6.2831853f * rnd();
        for (int k = 0; k < V; ++k) {
            const size_t c = (size_t)i * V + k;
            const float t = (float)k / (float)(V - 1);
            a.xyz[c] = x0 + 0.03f * std::sin(ph + 3.0f * t);
            a.xyz[(size_t)n * V + c] = 0.25f - 0.5f * t;
            a.xyz[2ull * n * V + c] = z0 - 0.05f * t;
        }
        a.sigma[i] = 0.2f + rnd();
        a.sigma[n + i] = 0.4f + rnd();
        a.sigma[2 * n + i] = 0.8f + rnd();
    }
    // strand 0: its last segment crosses the image from left to right
    const size_t last = (size_t)V - 1;
    a.xyz[last] = 2.0f;
    a.xyz[(size_t)n * V + last] = a.xyz[(size_t)n * V + last - 1];
    a.xyz[2ull * n * V + last] = a.xyz[2ull * n * V + last - 1];
    a.xyz[last - 1] = -2.0f;
    return a;
}

hair_material material() {
    hair_material m;
    std::memset(&m, 0, sizeof(m));
    m.eta = 1.55f;
    m.alpha = -0.035f;
    m.beta_m = 0.2f;
    m.beta_n = 0.3f;
    m.model = HAIR_MODEL_RTTRT;
    return m;
}

hair_camera camera(int W, int H) {
    hair_camera c;
    std::memset(&c, 0, sizeof(c));
    c.rot[0] = c.rot[4] = c.rot[8] = 1.0f;
    c.fx = c.fy = 300.0f;
    c.cx = 0.5f * W;
    c.cy = 0.5f * H;
    c.width = W;
    c.height = H;
    c.z_near = 0.01f;
    return c;
}

void lights(hair_light* l) {
    std::memset(l, 0, 2 * sizeof(hair_light));
    l[0].kind = 0;   // directional
    const float nrm = std::sqrt(0.5f * 0.5f + 0.6f * 0.6f + 0.62f * 0.62f);
    l[0].vec[0] = 0.5f / nrm; l[0].vec[1] = 0.6f / nrm; l[0].vec[2] = 0.62f / nrm;
    l[0].rgb[0] = l[0].rgb[1] = l[0].rgb[2] = 1.0f;
    l[1].kind = 1;   // point
    l[1].vec[0] = 0.3f; l[1].vec[1] = 0.3f; l[1].vec[2] = 0.0f;
    l[1].rgb[0] = l[1].rgb[1] = l[1].rgb[2] = 0.5f;
}

// Argument checking, valid on any context (host-only ones return HAIR_EDEVICE after it).
void check_arguments(hair_ctx* ctx, bool device) {
    const Asset a = make_asset(4, 3);
    const hair_material m = material();
    int32_t id = -1;
    EXPECT_RC(hair_upload(nullptr, a.n, a.V, a.xyz.data(), a.width.data(), a.sigma.data(), &m, nullptr, &id), HAIR_EINVAL);
    EXPECT_RC(hair_upload(ctx, a.n, 1, a.xyz.data(), a.width.data(), a.sigma.data(), &m, nullptr, &id), HAIR_EINVAL);
    EXPECT_RC(hair_upload(ctx, a.n, a.V, nullptr, a.width.data(), a.sigma.data(), &m, nullptr, &id), HAIR_EINVAL);
    std::vector<float> bad = a.xyz;
    bad[3] = NAN;
    EXPECT_RC(hair_upload(ctx, a.n, a.V, bad.data(), a.width.data(), a.sigma.data(), &m, nullptr, &id), HAIR_EINVAL);
    std::vector<float> w0 = a.width;
    w0[1] = 0.0f;
    EXPECT_RC(hair_upload(ctx, a.n, a.V, a.xyz.data(), w0.data(), a.sigma.data(), &m, nullptr, &id), HAIR_EINVAL);
    hair_material mb = m;
    mb.eta = 0.5f;
    EXPECT_RC(hair_upload(ctx, a.n, a.V, a.xyz.data(), a.width.data(), a.sigma.data(), &mb, nullptr, &id), HAIR_EINVAL);
    hair_camera cam = camera(64, 48);
    hair_light L[2];
    lights(L);
    hair_camera cb = cam;
    cb.width = 0;
    float dummy[4] = {0, 0, 0, 0};
    EXPECT_RC(hair_render(ctx, nullptr, 0, 0, &cb, L, 2, dummy, nullptr, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_render(ctx, nullptr, 0, 0, &cam, L, 0, dummy, nullptr, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_render(ctx, nullptr, 0, 0, &cam, L, HAIR_MAX_LIGHTS + 1, dummy, nullptr, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_render(ctx, nullptr, 0, 0, nullptr, L, 2, dummy, nullptr, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_render(ctx, nullptr, 0, 0, &cam, L, 2, nullptr, nullptr, nullptr), HAIR_EINVAL);
    hair_light lb[2];
    lights(lb);
    lb[0].vec[0] = NAN;
    EXPECT_RC(hair_render(ctx, nullptr, 0, 0, &cam, lb, 2, dummy, nullptr, nullptr), HAIR_EINVAL);
    hair_shadow sh = {8, 4, 0.02f};   // resolution below 16
    EXPECT_RC(hair_render_shadowed(ctx, nullptr, 0, 0, &cam, L, 2, &sh, dummy, nullptr, nullptr), HAIR_EINVAL);
    sh = {64, 9, 0.02f};              // more than 7 layers
    EXPECT_RC(hair_render_shadowed(ctx, nullptr, 0, 0, &cam, L, 2, &sh, dummy, nullptr, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_render_curved(ctx, nullptr, 0, 1, &cam, L, 2, 0, 4, dummy, nullptr, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_render_curved(ctx, nullptr, 0, 1, &cam, L, 2, 4, 17, dummy, nullptr, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_ws_create(nullptr, 0, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_ws_destroy(nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_ws_finish(nullptr, nullptr), HAIR_EINVAL);
    EXPECT_RC(hair_debug_segments(nullptr, 1, nullptr, nullptr), HAIR_EINVAL);
    EXPECT(hair_ws_estimate(1000, 256, 256, 0) > 0);
    EXPECT(hair_noalloc_scratch_bytes() == (64ull << 20));
    if (!device) {
        EXPECT_RC(hair_upload(ctx, a.n, a.V, a.xyz.data(), a.width.data(), a.sigma.data(), &m, nullptr, &id),
                  HAIR_EDEVICE);
        EXPECT_RC(hair_render(ctx, nullptr, 0, 0, &cam, L, 2, dummy, nullptr, nullptr), HAIR_ENOENT);
    }
}

// HIP runtime calls of the checker itself (buffers, copies): any failure ends the run.
void hip_ok(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        std::fprintf(stderr, "abi_check: %s: %s\n", what, hipGetErrorString(e));
        std::exit(2);
    }
}

template <class T>
T* dalloc(size_t n) {
    void* p = nullptr;
    hip_ok(hipMalloc(&p, sizeof(T) * (n ? n : 1)), "hipMalloc");
    hip_ok(hipMemset(p, 0, sizeof(T) * (n ? n : 1)), "hipMemset");
    return static_cast<T*>(p);
}

void check_device(hair_ctx* ctx) {
    const int W = 256, H = 256, n = 600, V = 9, S = V - 1;
    const Asset a = make_asset(n, V);
    const hair_material m = material();
    const hair_camera cam = camera(W, H);
    hair_light L[2];
    lights(L);
    int32_t id = -1;
    EXPECT_RC(hair_upload(ctx, a.n, a.V, a.xyz.data(), a.width.data(), a.sigma.data(), &m, nullptr, &id), HAIR_OK);
    uint64_t used = 0, budget = 0;
    EXPECT_RC(hair_ctx_memory(ctx, &used, &budget), HAIR_OK);
    EXPECT(used > 0 && budget >= used);
    hair_ws* ws = nullptr;
    EXPECT_RC(hair_ws_create(ctx, 0, &ws), HAIR_OK);
    float* img = dalloc<float>(4ull * W * H);
    float* img2 = dalloc<float>(4ull * W * H);
    std::vector<float> h1(4ull * W * H), h2(4ull * W * H);

    // strands: twice on one workspace (cold, then warm), bitwise equal; the long segment is
    // drawn in pieces, none culled
    hair_stats st1{}, st2{};
    EXPECT_RC(hair_render(ctx, ws, id, 0, &cam, L, 2, img, nullptr, &st1), HAIR_OK);
    EXPECT_RC(hair_render(ctx, ws, id, 0, &cam, L, 2, img2, nullptr, &st2), HAIR_OK);
    hip_ok(hipMemcpy(h1.data(), img, 4 * h1.size(), hipMemcpyDeviceToHost), "hipMemcpy");
    hip_ok(hipMemcpy(h2.data(), img2, 4 * h2.size(), hipMemcpyDeviceToHost), "hipMemcpy");
    EXPECT(st1.fragments > 0 && st1.fragments == st2.fragments);
    EXPECT(std::memcmp(h1.data(), h2.data(), 4 * h1.size()) == 0);
    EXPECT(st1.segments > (uint32_t)(n * S) && st1.segments_culled_long == 0);
    std::vector<int32_t> ri(6ull * st1.segments);
    std::vector<float> rf(3ull * st1.segments);
    EXPECT_RC(hair_debug_segments(ws, st1.segments, ri.data(), rf.data()), HAIR_OK);
    EXPECT_RC(hair_debug_segments(ws, st1.segments + 1, ri.data(), rf.data()), HAIR_EINVAL);
    const int T = ((W + 15) / 16) * ((H + 15) / 16);
    std::vector<uint32_t> ts(T + 1), segs(st1.pairs ? st1.pairs : 1);
    EXPECT_RC(hair_debug_bins(ws, T, ts.data(), (int64_t)st1.pairs, segs.data()), HAIR_OK);
    EXPECT(ts[T] == st1.pairs);

    // errors on a real context
    EXPECT_RC(hair_render(ctx, ws, id + 100, 0, &cam, L, 2, img, nullptr, nullptr), HAIR_ENOENT);
    EXPECT_RC(hair_render(ctx, ws, id, 3, &cam, L, 2, img, nullptr, nullptr), HAIR_ENOENT);
    int32_t lvl = -1;
    EXPECT_RC(hair_select_level(ctx, ws, id, &cam, 2.0f, nullptr, &lvl), HAIR_OK);
    EXPECT(lvl == 0);

    // thick-hair levels: 60 and 12 nested clusters
    const int K1 = 60, K2 = 12;
    std::vector<int32_t> assign(2ull * n);
    for (int s = 0; s < n; ++s) {
        assign[s] = s % K1;
        assign[(size_t)n + s] = (s % K1) % K2;
    }
    const int32_t ks[2] = {K1, K2};
    EXPECT_RC(hair_build_lod(ctx, id, 2, ks, assign.data(), nullptr), HAIR_OK);
    int32_t nl = 0, counts[4] = {0, 0, 0, 0}, sps = 0;
    EXPECT_RC(hair_lod_info(ctx, id, &nl, counts, 4, &sps), HAIR_OK);
    EXPECT(nl == 2 && counts[0] == n && counts[1] == K1 && counts[2] == K2 && sps == S);
    std::vector<float> centers(3ull * K2 * V), ahat(3ull * K2 * S), axes(2ull * K2 * S), sig(3ull * K2), r(K2);
    std::vector<int32_t> ntot(K2);
    EXPECT_RC(hair_get_lod(ctx, id, 2, K2, centers.data(), ahat.data(), axes.data(), ntot.data(), sig.data(), r.data()),
              HAIR_OK);
    EXPECT_RC(hair_get_lod(ctx, id, 2, K2 + 1, centers.data(), ahat.data(), axes.data(), ntot.data(), sig.data(),
                           r.data()),
              HAIR_EINVAL);
    EXPECT_RC(hair_set_lod(ctx, id, 2, K2, centers.data(), ahat.data(), axes.data(), ntot.data(), sig.data(), r.data(),
                           nullptr),
              HAIR_OK);
    float* d_axes = dalloc<float>(2ull * K1 * S);
    float* d_r = dalloc<float>(K1);
    float* d_sig = dalloc<float>(3ull * K1);
    for (int l = 1; l <= 2; ++l) {
        hair_stats st{};
        EXPECT_RC(hair_render(ctx, ws, id, l, &cam, L, 2, img, nullptr, &st), HAIR_OK);
        EXPECT(st.fragments > 0);
    }
    // backward at level 1, then its parameters written back unchanged
    float* d_rgba = dalloc<float>(4ull * W * H);
    std::vector<float> ones(4ull * W * H, 1.0f);
    hip_ok(hipMemcpy(d_rgba, ones.data(), 4 * ones.size(), hipMemcpyHostToDevice), "hipMemcpy");
    EXPECT_RC(hair_render_backward(ctx, ws, id, 1, &cam, L, 2, d_rgba, d_axes, d_r, d_sig, nullptr), HAIR_OK);
    EXPECT_RC(hair_render_backward(ctx, ws, id, 0, &cam, L, 2, d_rgba, d_axes, d_r, d_sig, nullptr), HAIR_EINVAL);
    {
        std::vector<float> c1(3ull * K1 * V), a1(3ull * K1 * S), x1(2ull * K1 * S), s1(3ull * K1), r1(K1);
        std::vector<int32_t> n1(K1);
        EXPECT_RC(hair_get_lod(ctx, id, 1, K1, c1.data(), a1.data(), x1.data(), n1.data(), s1.data(), r1.data()), HAIR_OK);
        hip_ok(hipMemcpy(d_axes, x1.data(), 4 * x1.size(), hipMemcpyHostToDevice), "hipMemcpy");
        hip_ok(hipMemcpy(d_r, r1.data(), 4 * r1.size(), hipMemcpyHostToDevice), "hipMemcpy");
        hip_ok(hipMemcpy(d_sig, s1.data(), 4 * s1.size(), hipMemcpyHostToDevice), "hipMemcpy");
        EXPECT_RC(hair_set_cluster_params(ctx, id, 1, d_axes, d_r, d_sig, nullptr), HAIR_OK);
        EXPECT_RC(hair_set_cluster_params(ctx, id, 1, nullptr, nullptr, nullptr, nullptr), HAIR_OK);
    }
    // shadows, curved centre lines
    hair_shadow sh = {128, 4, 0.02f};
    hair_stats st{};
    EXPECT_RC(hair_render_shadowed(ctx, ws, id, 0, &cam, L, 2, &sh, img, nullptr, &st), HAIR_OK);
    std::vector<float> tex(128ull * 128 * 8), grid(16);
    EXPECT_RC(hair_debug_dom(ws, 0, tex.data(), grid.data()), HAIR_OK);
    EXPECT_RC(hair_debug_dom(ws, 1, tex.data(), grid.data()), HAIR_EINVAL);   // point light: no map
    EXPECT_RC(hair_render_shadowed(ctx, ws, id, 1, &cam, L, 2, &sh, img, nullptr, &st), HAIR_OK);
    EXPECT_RC(hair_render_curved(ctx, ws, id, 1, &cam, L, 2, 4, 16, img, nullptr, &st), HAIR_OK);
    EXPECT_RC(hair_render_curved(ctx, ws, id, 0, &cam, L, 2, 4, 16, img, nullptr, &st), HAIR_EINVAL);

    // per-group LoD and mixed frames (plain and shadowed, with the deferred update)
    int32_t G = 0;
    EXPECT_RC(hair_lod_groups(ctx, id, &G), HAIR_OK);
    EXPECT(G == K2);
    int32_t* levels = dalloc<int32_t>((size_t)G * S);
    EXPECT_RC(hair_lod_init(ctx, ws, id, &cam, 3.0f, levels, nullptr), HAIR_OK);
    EXPECT_RC(hair_render_mixed(ctx, ws, id, &cam, L, 2, levels, 3.0f, img, nullptr, &st), HAIR_OK);
    EXPECT_RC(hair_render_mixed_shadowed(ctx, ws, id, &cam, L, 2, levels, 3.0f, &sh, img, nullptr, &st), HAIR_OK);
    std::vector<int32_t> hl((size_t)G * S, 1);
    hl[0] = 7;   // beyond the level count
    hip_ok(hipMemcpy(levels, hl.data(), 4 * hl.size(), hipMemcpyHostToDevice), "hipMemcpy");
    EXPECT_RC(hair_render_mixed(ctx, ws, id, &cam, L, 2, levels, 0.0f, img, nullptr, &st), HAIR_EINVAL);

    // asynchronous frames on two workspaces, then the allocation-free frame
    hair_ws* ws2 = nullptr;
    EXPECT_RC(hair_ws_create(ctx, 0, &ws2), HAIR_OK);
    EXPECT_RC(hair_render(ctx, ws2, id, 0, &cam, L, 2, img2, nullptr, nullptr), HAIR_OK);
    EXPECT_RC(hair_render_async(ctx, ws, id, 0, &cam, L, 2, img, nullptr), HAIR_OK);
    EXPECT_RC(hair_render_async(ctx, ws2, id, 0, &cam, L, 2, img2, nullptr), HAIR_OK);
    EXPECT_RC(hair_render(ctx, ws, id, 0, &cam, L, 2, img, nullptr, nullptr), HAIR_EINVAL);   // holds a frame
    hair_stats sa{}, sb{};
    EXPECT_RC(hair_ws_finish(ws, &sa), HAIR_OK);
    EXPECT_RC(hair_ws_finish(ws2, &sb), HAIR_OK);
    EXPECT(sa.fragments == st1.fragments && sb.fragments == st1.fragments);
    EXPECT_RC(hair_ws_finish(ws, &sa), HAIR_OK);   // nothing held
    const hair_camera small = camera(64, 64);
    EXPECT_RC(hair_render_noalloc(ctx, id, 0, &small, L, 2, img, nullptr, &st), HAIR_OK);

    // workspace limits: a limit below the frame's needs fails without writing, trim frees
    uint64_t held = 0, maxb = 0;
    EXPECT_RC(hair_ws_memory(ws2, &held, &maxb), HAIR_OK);
    EXPECT(held > 0);
    EXPECT_RC(hair_ws_trim(ws2), HAIR_OK);
    EXPECT_RC(hair_ws_set_limit(ws2, 4096), HAIR_OK);
    EXPECT_RC(hair_render(ctx, ws2, id, 0, &cam, L, 2, img2, nullptr, nullptr), HAIR_ENOMEM);
    EXPECT_RC(hair_ws_set_limit(ws2, 0), HAIR_OK);
    EXPECT_RC(hair_render(ctx, ws2, id, 0, &cam, L, 2, img2, nullptr, nullptr), HAIR_OK);

    // composited fragment lists of a few pixels
    const int64_t cap = 64 * 1536;
    std::vector<uint32_t> cnt(64), keys(cap), sids(cap);
    std::vector<float> al(cap), ho(cap);
    EXPECT_RC(hair_debug_fragments(ctx, ws, id, 0, &cam, L, 2, 124, 124, 8, 8, cnt.data(), cap, keys.data(), sids.data(),
                                   al.data(), ho.data(), nullptr),
              HAIR_OK);
    double rate = 0.0;
    EXPECT_RC(hair_debug_issue_rate(ctx, 0, 64, &rate), HAIR_OK);
    EXPECT(rate > 0.0);

    EXPECT_RC(hair_release(ctx, id), HAIR_OK);
    EXPECT_RC(hair_release(ctx, id), HAIR_ENOENT);
    EXPECT_RC(hair_ws_destroy(ws2), HAIR_OK);
    EXPECT_RC(hair_ws_destroy(ws), HAIR_OK);
    hip_ok(hipFree(levels), "hipFree");
    hip_ok(hipFree(d_rgba), "hipFree");
    hip_ok(hipFree(d_axes), "hipFree");
    hip_ok(hipFree(d_r), "hipFree");
    hip_ok(hipFree(d_sig), "hipFree");
    hip_ok(hipFree(img), "hipFree");
    hip_ok(hipFree(img2), "hipFree");
}

}  // namespace

int main(int argc, char** argv) {
    int device = -2;
    for (int i = 1; i < argc; ++i) {
        if (!std::strcmp(argv[i], "--host-only")) device = -1;
        else if (!std::strcmp(argv[i], "--device") && i + 1 < argc) device = std::atoi(argv[++i]);
    }
    if (device < -1) {
        std::fprintf(stderr, "usage: abi_check --host-only | --device N\n");
        return 2;
    }
    EXPECT(hair_version() > 0);
    EXPECT(hair_last_error() != nullptr);
    EXPECT_RC(hair_ctx_create(-2, 0, nullptr), HAIR_EINVAL);
    hair_ctx* ctx = nullptr;
    EXPECT_RC(hair_ctx_create(device, 0, &ctx), HAIR_OK);
    if (ctx) {
        check_arguments(ctx, device >= 0);
        if (device >= 0) check_device(ctx);
        EXPECT_RC(hair_ctx_destroy(ctx), HAIR_OK);
    }
    std::printf("abi_check: %d checks, %d failed (%s)\n", g_checks, g_fail, device >= 0 ? "device" : "host-only");
    return g_fail ? 1 : 0;
}
