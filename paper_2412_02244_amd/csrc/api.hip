// C ABI of libekm: argument checks, workspace, and the per-iteration
// pipeline  A1 centroid tree -> A2 leaf candidates -> A3/A4 assignment with
// fused exact accumulation -> A5 refinement (one pass of Algorithm 1's loop).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>

#include "ekm_internal.hpp"
#include "finalize.hpp"

namespace ekm {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

bool hip_ok(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return true;
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

int64_t assign_blocks(km_ctx *ctx);

static int ceil_log2(int64_t v)
{
    int h = 0;
    while (((int64_t)1 << h) < v)
        ++h;
    return h;
}

static km_status check_config(const km_config *cfg, int64_t n, int64_t k)
{
    if (!cfg) {
        set_error("null km_config");
        return KM_ERR_INVALID;
    }
    if (cfg->d != 2 && cfg->d != 3) {
        set_error("d must be 2 or 3");
        return KM_ERR_INVALID;
    }
    if (cfg->point_dtype != KM_F32 && cfg->point_dtype != KM_F64) {
        set_error("point_dtype must be KM_F32 or KM_F64");
        return KM_ERR_INVALID;
    }
    if (cfg->algo != KM_BRUTE && cfg->algo != KM_INDEXED) {
        set_error("algo must be KM_BRUTE or KM_INDEXED");
        return KM_ERR_INVALID;
    }
    if (n < 1 || n >= ((int64_t)1 << 31)) {
        set_error("n must be in [1, 2^31)");
        return KM_ERR_INVALID;
    }
    if (k < 1 || k > n) {
        set_error("k must be in [1, n]");
        return KM_ERR_INVALID;
    }
    if (k > ((int64_t)1 << 20)) {
        set_error("k must be at most 2^20");
        return KM_ERR_UNSUPPORTED;
    }
    int f = cfg->leaf_size;
    if (f != 0 && (f < 8 || f > MAX_LEAF || (f & (f - 1)))) {
        set_error("leaf_size must be 0 or a power of two in [8, 64]");
        return KM_ERR_INVALID;
    }
    int t = cfg->cand_tile;
    if (cfg->algo == KM_INDEXED && t != 0 && (t < 1 || t > GROUP_LEAVES)) {
        set_error("cand_tile (indexed: leaves sharing one candidate list) must be 0 or in [1, 8]");
        return KM_ERR_INVALID;
    }
    if (cfg->algo == KM_BRUTE && t != 0 && (t < 64 || t > 2048)) {
        set_error("cand_tile (brute: centroids per LDS tile) must be 0 or in [64, 2048]");
        return KM_ERR_INVALID;
    }
    if (cfg->algo == KM_INDEXED && cfg->point_dtype != KM_F32) {
        set_error("KM_INDEXED needs FP32 points (FP64 points run with KM_BRUTE)");
        return KM_ERR_UNSUPPORTED;
    }
    return KM_OK;
}

// ------------------------------------------------------------ memory model
// The device workspace of a context, buffer by buffer, from the counts that
// size them (the memory estimation of Eq. (10)-(11), adapted to this
// library's buffers): per point, per leaf, per leaf group, per centroid and
// per centroid-tree node.  ws_bytes is exact for given counts; the counts of
// leaves and groups are only known once the points are sorted, so the
// estimate takes cells half full on average, the paper's assumption: a
// group cell (at most G f points) holds G f / 2 points, cut into leaves of
// f points (default leaves), or a leaf cell (at most f points) holds f / 2
// points (KM_FLAG_CELL_LEAVES, and the leaf cuts of the brute path).
struct WsCounts {
    int64_t n = 0, k = 0, B = 1;
    int64_t L = 0, groups = 0;  // leaves, leaf groups
    int64_t nodes = 0, pair_blocks = 0; // centroid-tree nodes and inter-bound pair-scan workgroups
    int64_t kmax = 0;                   // centroids of the largest cloud
};

// The workspace in the order the build allocates it: `build` (cloud tables,
// sort keys and scratch, kept for the centroid sort, and the SoA points:
// known from n alone), `rest` (leaves, per-step buffers, centroid trees and
// per-leaf state: needs the leaf count), `groups` (leaf groups and their
// statistics rows: needs the group count) and the statistics rows of a run.
struct WsParts {
    size_t build = 0, rest = 0, groups = 0, hist = 0;
    size_t total() const { return build + rest + groups + hist; }
};

static WsParts ws_parts(const km_config *cfg, const WsCounts &c)
{
    auto al = [](int64_t count, size_t elem) { return alloc_size((size_t)(count > 0 ? count : 0), elem); };
    const int d = cfg->d;
    const size_t es = cfg->point_dtype == KM_F32 ? 4 : 8;
    const bool indexed = cfg->algo == KM_INDEXED;
    const bool leaf_state = indexed && cfg->point_dtype == KM_F32;
    const int64_t n = c.n, k = c.k, L = c.L;
    const int64_t hist = (int64_t)radix_scratch_words(n);
    WsParts p;
    p.build = 2 * al(c.B + 1, 8) + al(c.B + 1, scan_record_bytes()) + al(c.B, sizeof(Grid)) + 4 * al(n, 4) +
              al(hist, 4) + al((int64_t)scan_scratch_words(hist > n ? hist : n), 4) + al(n * d, es);
    p.rest = al(L + 1, 4);
    if (leaf_state)
        p.rest += al(2 * L, 16) + al(L * d * 2, 8) + al(L, 4);
    p.rest += al(n, 4) + al(k, 16) + al(k, 4) + al(1, 4) + al(k * d * 2, 8) + al(k, 4);
    p.rest += al(sse_blocks(n), 8) + al(NSTAT, 8) + al(1, 8) + al(k * d, 8);
    p.rest += al(FIN_MAX_STAT_WG * (NSTAT + 1), 8) + al(1, 4); // statistics hand-over (finalize.hpp)
    if (indexed) // centroid trees, inter bounds, per-leaf state
        p.rest += al(k, 16) + 2 * al(c.nodes, 16) + al(c.B, sizeof(TreeArgs)) +
                  al(c.pair_blocks * PAIR_WAVES, sizeof(PairItem)) +
                  3 * al(L, 4) + al(1, 4) + 3 * al(k, 4) + al(1, 4) + al(k * d, 8);
    p.rest += al(CTL_N, 4);
    const int64_t nblk = indexed ? (c.groups + main_waves(d) - 1) / main_waves(d) + heavy_blocks(c.kmax)
                                 : (n + 255) / 256;
    if (leaf_state)
        p.groups = al(c.groups + 1, 4) + al(2 * c.groups, 16) + 2 * al(c.groups, 4);
    p.groups += al(nblk * NSTAT, 8);
    p.hist = (size_t)HIST_ROWS * (NSTAT + 1) * 8;
    return p;
}

static size_t ws_bytes(const km_config *cfg, const WsCounts &c) { return ws_parts(cfg, c).total(); }

// Estimated counts for B clouds (pt_off / c_off, host) at leaf size f and G
// leaves per group.
static WsCounts ws_estimate(const km_config *cfg, int B, const int64_t *pt_off, const int64_t *c_off, int f, int G)
{
    WsCounts c;
    c.n = pt_off[B];
    c.k = c_off[B];
    c.B = B;
    const bool packed =
        cfg->algo == KM_INDEXED && cfg->point_dtype == KM_F32 && !(cfg->flags & KM_FLAG_CELL_LEAVES);
    bool small = true; // every cloud's tree is built in LDS, with the pair scan of the inter bound
    for (int b = 0; b < B; ++b) {
        const int64_t nb = pt_off[b + 1] - pt_off[b], kb = c_off[b + 1] - c_off[b];
        if (packed) {
            const int64_t cells = (2 * nb + (int64_t)G * f - 1) / ((int64_t)G * f); // half-full group cells
            c.groups += cells;
            c.L += cells * (((int64_t)G * f / 2 + f - 1) / f);
        } else {
            const int64_t leaves = (2 * nb + f - 1) / f; // half-full leaf cells
            c.L += leaves;
            c.groups += (leaves + G - 1) / G;
        }
        TreeArgs T;
        tree_layout(kb, T);
        c.nodes += T.nnodes;
        c.kmax = kb > c.kmax ? kb : c.kmax;
        small = small && kb <= TREE_SMALL_K;
    }
    if (cfg->algo == KM_INDEXED && small)
        c.pair_blocks = pair_plan(c_off, B, nullptr);
    return c;
}

static size_t model_bytes(const km_config *cfg, int B, const int64_t *pt_off, const int64_t *c_off, int f, int G)
{
    return ws_bytes(cfg, ws_estimate(cfg, B, pt_off, c_off, f, G));
}

size_t ctx_bytes_after_counts(const km_ctx *ctx, int64_t L, int64_t groups, bool with_groups)
{
    WsCounts c = ws_estimate(&ctx->cfg, ctx->B, ctx->h_pt_off.data(), ctx->h_c_off.data(), ctx->f, ctx->G);
    c.L = L;
    c.groups = groups;
    const WsParts p = ws_parts(&ctx->cfg, c);
    return p.rest + (with_groups ? p.groups : 0);
}

// Device bytes a context holds.
static size_t ctx_device_bytes(const km_ctx *ctx)
{
    return ctx->mem.bytes + (size_t)ctx->hist_cap * (NSTAT + 1) * sizeof(int64_t);
}

// Leaves per group for a configuration (cand_tile, else the default).
static int default_groups(const km_config *cfg)
{
    if (cfg->algo == KM_INDEXED && cfg->cand_tile)
        return cfg->cand_tile;
    return cfg->d == 2 && !(cfg->flags & KM_FLAG_CELL_LEAVES) ? DEFAULT_G_2D : GROUP_LEAVES;
}

// Leaf size: cfg->leaf_size, or with a workspace limit on the indexed path
// the smallest power of two in [8, 64] whose modelled workspace fits (the
// memory-tunable index of Eq. (12): the finest index the memory allows), or
// 64 (0 if nothing fits).
static int choose_leaf_size(const km_config *cfg, int B, const int64_t *pt_off, const int64_t *c_off)
{
    if (cfg->leaf_size)
        return cfg->leaf_size;
    if (cfg->algo != KM_INDEXED || cfg->workspace_limit_bytes <= 0)
        return 64;
    const int G = default_groups(cfg);
    for (int f = 8; f <= MAX_LEAF; f *= 2)
        if (model_bytes(cfg, B, pt_off, c_off, f, G) <= (size_t)cfg->workspace_limit_bytes)
            return f;
    return 0;
}

static km_status alloc_fail(km_ctx *ctx)
{
    (void)ctx;
    set_error("device allocation failed");
    return KM_ERR_OOM;
}

// Host statistics from a row of NSTAT counters followed by the SSE bits.
static void fill_stats(const km_ctx *ctx, const int64_t *h, km_iter_stats *stats)
{
    stats->n_changed = h[ST_CHANGED];
    stats->dist_evals = h[ST_EVALS];
    stats->brute_evals = ctx->n * ctx->k;
    stats->single_cand_points = h[ST_SINGLE];
    stats->rechecked = h[ST_RECHECK];
    stats->cand_total = h[ST_CANDS];
    stats->leaves = ctx->cfg.algo == KM_INDEXED ? ctx->L : 0;
    double sse;
    memcpy(&sse, h + NSTAT, sizeof(double));
    stats->sse = (ctx->cfg.flags & KM_FLAG_SSE) ? sse : 0.0;
    stats->inter_leaf_points = h[ST_KEEP_LEAF_PTS];
    stats->inter_points = h[ST_KEEP_PTS];
    stats->fallback_points = h[ST_FALLBACK_PTS];
    stats->deferred_leaves = h[ST_DEFERRED];
    stats->group_overflows = h[ST_GROUP_OVF];
    stats->groups_skipped = h[ST_GROUP_SKIP];
    stats->region_points = h[ST_REGION_PTS];
}

// One step's launches: A1 tree (+ inter bounds), A2-A5 assignment passes,
// objective, refinement.  ev: KM_NPHASE + 1 events to record at the phase
// boundaries, or null.  pos: the step's place in its sequence of launches
// (a context's single steps, or the steps of one graph); the large-k
// centroid tree re-sorts at every TREE_RESORT-th, the first included.
static km_status step_body(km_ctx *ctx, const double *c_in, double *c_out, int32_t *assign_out, hipEvent_t *ev,
                           int64_t pos)
{
    auto mark = [&](int i) {
        if (ev)
            hipEventRecord(ev[i], ctx->stream);
    };
    km_status s;
    mark(KM_PHASE_TREE);
    if (ctx->cfg.point_dtype == KM_F32 && (s = build_centroid_tree(ctx, c_in, pos % TREE_RESORT == 0)) != KM_OK)
        return s;
    mark(KM_PHASE_ASSIGN);
    if ((s = run_assign(ctx, c_in, ev ? ev[KM_PHASE_DEFERRED] : nullptr)) != KM_OK)
        return s;
    mark(KM_PHASE_UPDATE);
    const bool want_sse = (ctx->cfg.flags & KM_FLAG_SSE) != 0;
    if (want_sse && (s = run_sse(ctx, c_in)) != KM_OK)
        return s;
    if ((s = run_finalize(ctx, c_in, c_out, nullptr, want_sse)) != KM_OK)
        return s;
    mark(KM_NPHASE);
    if (assign_out && (s = scatter_assignment(ctx, assign_out)) != KM_OK)
        return s;
    return KM_OK;
}

// A step with KM_FLAG_TIMING events when the context records them: the
// step's events join the record only when the step succeeded.
static km_status timed_step(km_ctx *ctx, const double *c_in, double *c_out, int32_t *assign_out, int64_t pos)
{
    const bool timing = (ctx->cfg.flags & KM_FLAG_TIMING) != 0;
    if (!timing)
        return step_body(ctx, c_in, c_out, assign_out, nullptr, pos);
    std::array<hipEvent_t, KM_NPHASE + 1> ev{};
    int have = 0;
    for (auto &e : ev) {
        if (!ctx->ev_pool.empty()) {
            e = ctx->ev_pool.back();
            ctx->ev_pool.pop_back();
        } else if (!hip_ok(hipEventCreate(&e), "hipEventCreate")) {
            break;
        }
        ++have;
    }
    km_status s = have == KM_NPHASE + 1 ? step_body(ctx, c_in, c_out, assign_out, ev.data(), pos) : KM_ERR_HIP;
    if (s == KM_OK)
        ctx->ev_steps.push_back(ev);
    else
        for (int i = 0; i < have; ++i)
            ctx->ev_pool.push_back(ev[i]);
    return s;
}

// kmeans_run's chunk of RUN_CHUNK steps on centroid array c (the context's
// own), captured once into a graph (on a private stream; launched on the
// context's stream).
// Returns false when capture is not possible; the caller then launches the
// steps one by one, with the same result.
static bool chunk_graph(km_ctx *ctx, double *c)
{
    if (ctx->chunk_failed)
        return false;
    if (ctx->chunk_exec && ctx->chunk_c == c)
        return true;
    if (ctx->chunk_exec) {
        (void)hipGraphExecDestroy(ctx->chunk_exec);
        ctx->chunk_exec = nullptr;
    }
    if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        ctx->cap_stream = nullptr;
        ctx->chunk_failed = 1;
        (void)hipGetLastError();
        return false;
    }
    hipStream_t saved = ctx->stream;
    ctx->stream = ctx->cap_stream;
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        for (int i = 0; ok && i < RUN_CHUNK; ++i)
            ok = step_body(ctx, c, c, nullptr, nullptr, i) == KM_OK;
        ok = hipStreamEndCapture(ctx->cap_stream, &g) == hipSuccess && ok && g;
    }
    ctx->stream = saved;
    if (ok)
        ok = hipGraphInstantiate(&ctx->chunk_exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g)
        (void)hipGraphDestroy(g);
    if (!ok) {
        ctx->chunk_exec = nullptr;
        ctx->chunk_failed = 1;
        (void)hipGetLastError();
        return false;
    }
    ctx->chunk_c = c;
    return true;
}

} // namespace ekm

using namespace ekm;

extern "C" {

size_t kmeans_workspace_bytes(const km_config *cfg, int64_t n, int64_t k)
{
    if (check_config(cfg, n, k) != KM_OK)
        return 0;
    const int64_t pt_off[2] = {0, n}, c_off[2] = {0, k};
    const int f = choose_leaf_size(cfg, 1, pt_off, c_off);
    return model_bytes(cfg, 1, pt_off, c_off, f ? f : MAX_LEAF, default_groups(cfg));
}

km_status kmeans_context_info(const km_ctx *ctx, km_ctx_info *info)
{
    if (!ctx || !info) {
        set_error("kmeans_context_info: null argument");
        return KM_ERR_INVALID;
    }
    info->device_bytes = (int64_t)ctx_device_bytes(ctx);
    info->leaf_size = ctx->f;
    info->leaves_per_group = ctx->G;
    info->leaves = ctx->L;
    info->groups = ctx->ngroups;
    info->allocations = (int64_t)ctx->mem.ptrs.size() + (ctx->stat_hist ? 1 : 0);
    WsCounts c = ws_estimate(&ctx->cfg, ctx->B, ctx->h_pt_off.data(), ctx->h_c_off.data(), ctx->f, ctx->G);
    info->model_bytes = (int64_t)ws_bytes(&ctx->cfg, c);
    c.L = ctx->L;
    c.groups = ctx->ngroups;
    info->model_bytes_actual_counts = (int64_t)ws_bytes(&ctx->cfg, c);
    return KM_OK;
}

const char *kmeans_last_error(void) { return g_error.c_str(); }

// Elapsed times of every recorded step, [step][phase]; nothing changes on error.
static km_status recorded_times(km_ctx *ctx, std::vector<double> &out)
{
    if (!hip_ok(hipStreamSynchronize(ctx->stream), "phase times: hipStreamSynchronize"))
        return KM_ERR_HIP;
    out.assign(ctx->ev_steps.size() * KM_NPHASE, 0.0);
    for (size_t s = 0; s < ctx->ev_steps.size(); ++s) {
        const auto &ev = ctx->ev_steps[s];
        for (int p = 0; p < KM_NPHASE; ++p) {
            float t = 0.0f;
            if (!hip_ok(hipEventElapsedTime(&t, ev[p], ev[p + 1]), "phase times: hipEventElapsedTime"))
                return KM_ERR_HIP;
            out[s * KM_NPHASE + p] = t;
        }
    }
    return KM_OK;
}

static void release_recorded(km_ctx *ctx)
{
    for (auto &ev : ctx->ev_steps)
        for (auto e : ev)
            ctx->ev_pool.push_back(e);
    ctx->ev_steps.clear();
}

km_status kmeans_phase_times(km_ctx *ctx, double *ms, int64_t *steps)
{
    if (!ctx || !ms || !steps) {
        set_error("kmeans_phase_times: null argument");
        return KM_ERR_INVALID;
    }
    std::vector<double> t;
    km_status s = recorded_times(ctx, t);
    if (s != KM_OK)
        return s;
    for (int p = 0; p < KM_NPHASE; ++p)
        ms[p] = 0.0;
    for (size_t i = 0; i < t.size(); ++i)
        ms[i % KM_NPHASE] += t[i];
    *steps = (int64_t)ctx->ev_steps.size();
    release_recorded(ctx);
    return KM_OK;
}

km_status kmeans_step_times(km_ctx *ctx, double *ms, int64_t cap, int64_t *steps)
{
    if (!ctx || !steps || cap < 0 || (cap > 0 && !ms)) {
        set_error("kmeans_step_times: invalid argument");
        return KM_ERR_INVALID;
    }
    std::vector<double> t;
    km_status s = recorded_times(ctx, t);
    if (s != KM_OK)
        return s;
    const int64_t n = (int64_t)ctx->ev_steps.size();
    for (int64_t i = 0; i < (n < cap ? n : cap) * KM_NPHASE; ++i)
        ms[i] = t[i];
    *steps = n;
    release_recorded(ctx);
    return KM_OK;
}

km_status kmeans_destroy(km_ctx *ctx)
{
    if (!ctx)
        return KM_OK;
    hipStreamSynchronize(ctx->stream);
    for (auto &ev : ctx->ev_steps)
        for (auto e : ev)
            hipEventDestroy(e);
    for (auto e : ctx->ev_pool)
        hipEventDestroy(e);
    for (void *p : ctx->mem.ptrs)
        hipFree(p);
    if (ctx->host_stat)
        hipHostFree(ctx->host_stat);
    if (ctx->host_ctl)
        hipHostFree(ctx->host_ctl);
    for (auto e : ctx->chunk_ev)
        if (e)
            hipEventDestroy(e);
    if (ctx->stat_hist)
        hipFree(ctx->stat_hist);
    if (ctx->chunk_exec)
        hipGraphExecDestroy(ctx->chunk_exec);
    if (ctx->cap_stream)
        hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return KM_OK;
}

// Context over B clouds (B = 1: kmeans_init) with point / centroid offsets
// pt_off / c_off ([B + 1], host), already validated.
static km_status init_context(km_ctx **out, const km_config *cfg, const void *points, int B, const int64_t *pt_off,
                              const int64_t *c_off, void *stream, bool capture_chunk = true, int f_retry = 0)
{
    const int64_t n = pt_off[B], k = c_off[B];
    const int f = f_retry ? f_retry : choose_leaf_size(cfg, B, pt_off, c_off);
    const int G = default_groups(cfg);
    if (cfg->workspace_limit_bytes > 0 &&
        (f == 0 || model_bytes(cfg, B, pt_off, c_off, f, G) > (size_t)cfg->workspace_limit_bytes)) {
        set_error("kmeans_init: the modelled workspace (" +
                  std::to_string(model_bytes(cfg, B, pt_off, c_off, f ? f : MAX_LEAF, G)) +
                  " bytes at the largest leaf size) exceeds workspace_limit_bytes");
        return KM_ERR_OOM;
    }
    static std::once_flag once;
    static hipError_t setup_err = hipSuccess;
    std::call_once(once, [] { setup_err = tree_setup(); });
    if (!hip_ok(setup_err, "kmeans_init: kernel setup"))
        return KM_ERR_HIP;

    km_ctx *ctx = new km_ctx();
    ctx->cfg = *cfg;
    ctx->n = n;
    ctx->k = k;
    ctx->d = cfg->d;
    ctx->f = f;
    ctx->G = G;
    ctx->tile = cfg->algo == KM_BRUTE && cfg->cand_tile ? cfg->cand_tile : 1024;
    ctx->stream = (hipStream_t)stream;
    ctx->small_lists = (cfg->flags & KM_FLAG_SMALL_LISTS) ? 1 : 0;
    {
        int64_t kmax = 0;
        for (int b = 0; b < B; ++b)
            kmax = c_off[b + 1] - c_off[b] > kmax ? c_off[b + 1] - c_off[b] : kmax;
        ctx->heavy_wgs = heavy_blocks(kmax);
    }
    hipGetDevice(&ctx->device);
    hipStream_t st = ctx->stream;
    km_status s;
    ctx->B = B;
    ctx->h_pt_off.assign(pt_off, pt_off + B + 1);
    ctx->h_c_off.assign(c_off, c_off + B + 1);
    // the buffers of the index build, in one allocation (their sizes follow from n)
    if (!ctx_arena(ctx, ws_parts(cfg, ws_estimate(cfg, B, pt_off, c_off, f, G)).build)) {
        kmeans_destroy(ctx);
        return alloc_fail(nullptr);
    }
    ctx->pt_off = ctx_alloc<int64_t>(ctx, B + 1);
    ctx->c_off = ctx_alloc<int64_t>(ctx, B + 1);
    if (!ctx->pt_off || !ctx->c_off) {
        kmeans_destroy(ctx);
        return alloc_fail(nullptr);
    }
    if (!hip_ok(hipMemcpyAsync(ctx->pt_off, pt_off, (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st),
                "hipMemcpyAsync") ||
        !hip_ok(hipMemcpyAsync(ctx->c_off, c_off, (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st),
                "hipMemcpyAsync")) {
        kmeans_destroy(ctx);
        return KM_ERR_HIP;
    }

    s = build_leaves(ctx, points);
    if (s != KM_OK) {
        kmeans_destroy(ctx);
        return s;
    }
    const int64_t L = ctx->L;
    ctx->a = ctx_alloc<int32_t>(ctx, n);
    ctx->c32 = ctx_alloc<float4>(ctx, k);
    ctx->cval = ctx_alloc<int32_t>(ctx, k);
    ctx->cerr = ctx_alloc<float>(ctx, 1);
    ctx->acc = ctx_alloc<int64_t>(ctx, (size_t)k * ctx->d * 2);
    ctx->cnt = ctx_alloc<int32_t>(ctx, k);
    ctx->nblk_stat = assign_blocks(ctx);
    ctx->stat_part = ctx_alloc_groups<int64_t>(ctx, (size_t)ctx->nblk_stat * NSTAT);
    ctx->fin_part = ctx_alloc<int64_t>(ctx, (size_t)FIN_MAX_STAT_WG * (NSTAT + 1));
    ctx->fin_ticket = ctx_alloc<int32_t>(ctx, 1);
    ctx->nblk_sse = sse_blocks(n);
    ctx->sse_part = ctx_alloc<double>(ctx, ctx->nblk_sse);
    ctx->stat_out = ctx_alloc<int64_t>(ctx, NSTAT);
    ctx->sse_out = ctx_alloc<double>(ctx, 1);
    ctx->c_run = ctx_alloc<double>(ctx, (size_t)k * ctx->d);
    if (hipMalloc((void **)&ctx->stat_hist, (size_t)HIST_ROWS * (NSTAT + 1) * sizeof(int64_t)) == hipSuccess)
        ctx->hist_cap = HIST_ROWS;
    else
        ctx->stat_hist = nullptr;
    if (!ctx->a || !ctx->c32 || !ctx->cval || !ctx->cerr || !ctx->acc || !ctx->cnt || !ctx->stat_part ||
        !ctx->fin_part || !ctx->fin_ticket ||
        !ctx->sse_part || !ctx->stat_out || !ctx->sse_out || !ctx->c_run || !ctx->stat_hist) {
        kmeans_destroy(ctx);
        return alloc_fail(nullptr);
    }
    if (cfg->algo == KM_INDEXED) {
        // one tree per cloud, in concatenated arrays (tree positions local,
        // ids global), and the wave items of the inter-bound pair scan
        ctx->h_trees.assign(B, TreeArgs{});
        int64_t nn = 0;
        for (int b = 0; b < B; ++b) {
            TreeArgs &T = ctx->h_trees[b];
            T.k = c_off[b + 1] - c_off[b];
            T.c0 = c_off[b];
            tree_layout(T.k, T);
            nn += T.nnodes;
        }
        std::vector<PairItem> pairs;
        if (small_trees(ctx)) {
            ctx->npair_blocks = pair_plan(c_off, B, &pairs);
            ctx->tree_kcap = small_tree_cap(c_off, B);
        }
        float4 *cs = ctx_alloc<float4>(ctx, k), *nlo = ctx_alloc<float4>(ctx, nn), *nhi = ctx_alloc<float4>(ctx, nn);
        ctx->trees = ctx_alloc<TreeArgs>(ctx, B);
        ctx->pair_items = ctx_alloc<PairItem>(ctx, pairs.size());
        if (!cs || !nlo || !nhi || !ctx->trees || (!pairs.empty() && !ctx->pair_items)) {
            kmeans_destroy(ctx);
            return alloc_fail(nullptr);
        }
        for (int b = 0, no = 0; b < B; ++b) {
            TreeArgs &T = ctx->h_trees[b];
            T.cs = cs + T.c0;
            T.node_lo = nlo + no;
            T.node_hi = nhi + no;
            no += (int)T.nnodes;
        }
        ctx->tree = ctx->h_trees[0];
        // the large-k tree keeps its last order between sorts: start from the identity
        std::vector<float4> order;
        if (!small_trees(ctx)) {
            order.resize((size_t)k);
            for (int64_t j = 0; j < k; ++j) {
                const int32_t id = (int32_t)j;
                float w;
                memcpy(&w, &id, sizeof(w)); // the id's bits, as the tree stores it
                order[(size_t)j] = make_float4(0.0f, 0.0f, 0.0f, w);
            }
        }
        if (!hip_ok(hipMemcpyAsync(ctx->trees, ctx->h_trees.data(), B * sizeof(TreeArgs), hipMemcpyHostToDevice, st),
                    "hipMemcpyAsync") ||
            (!order.empty() && !hip_ok(hipMemcpyAsync(cs, order.data(), order.size() * sizeof(float4),
                                                      hipMemcpyHostToDevice, st),
                                       "hipMemcpyAsync")) ||
            (!pairs.empty() && !hip_ok(hipMemcpyAsync(ctx->pair_items, pairs.data(), pairs.size() * sizeof(PairItem),
                                                      hipMemcpyHostToDevice, st),
                                       "hipMemcpyAsync")) ||
            !hip_ok(hipStreamSynchronize(st), "hipStreamSynchronize")) { // the host vectors go out of scope
            kmeans_destroy(ctx);
            return KM_ERR_HIP;
        }
        ctx->leaf_own = ctx_alloc<int32_t>(ctx, L);
        ctx->leaf_r = ctx_alloc<float>(ctx, L);
        ctx->heavy = ctx_alloc<int32_t>(ctx, L);
        ctx->heavy_cnt = ctx_alloc<int32_t>(ctx, 1);
        ctx->cb_s = ctx_alloc<unsigned>(ctx, k);
        ctx->cb_hi = ctx_alloc<float>(ctx, k);
        ctx->drift = ctx_alloc<float>(ctx, k);
        ctx->drift_max = ctx_alloc<unsigned>(ctx, 1);
        ctx->c_prev = ctx_alloc<double>(ctx, (size_t)k * ctx->d);
        ctx->group_parts = ctx_alloc_groups<int32_t>(ctx, ctx->ngroups);
        if (!ctx->leaf_own || !ctx->leaf_r || !ctx->heavy || !ctx->heavy_cnt || !ctx->cb_s ||
            !ctx->cb_hi || !ctx->drift || !ctx->drift_max || !ctx->c_prev || !ctx->group_parts) {
            kmeans_destroy(ctx);
            return alloc_fail(nullptr);
        }
        if (!hip_ok(hipMemsetD32Async(ctx->leaf_own, OWN_NONE, L, st), "hipMemsetD32Async") ||
            !hip_ok(hipMemsetD32Async(ctx->leaf_r, 0x7f800000, L, st), "hipMemsetD32Async") || // +inf
            !hip_ok(hipMemsetAsync(ctx->heavy, 0, L * sizeof(int32_t), st), "hipMemsetAsync") ||
            !hip_ok(hipMemsetAsync(ctx->drift_max, 0, sizeof(unsigned), st), "hipMemsetAsync") ||
            !hip_ok(hipMemsetAsync(ctx->heavy_cnt, 0, sizeof(int32_t), st), "hipMemsetAsync") ||
            !hip_ok(hipMemsetAsync(ctx->group_parts, 0, ctx->ngroups * sizeof(int32_t), st), "hipMemsetAsync")) {
            kmeans_destroy(ctx);
            return KM_ERR_HIP;
        }
    }
    ctx->ctl = ctx_alloc<int32_t>(ctx, CTL_N);
    if (!ctx->ctl || !hip_ok(hipMemsetAsync(ctx->ctl, 0, CTL_N * sizeof(int32_t), st), "hipMemsetAsync") ||
        set_ctl(ctx, 0, 0, 1) != KM_OK) {
        kmeans_destroy(ctx);
        return alloc_fail(nullptr);
    }
    if (hipHostMalloc((void **)&ctx->host_ctl, (RUN_AHEAD + 1) * CTL_N * sizeof(int32_t), hipHostMallocDefault) !=
        hipSuccess) {
        ctx->host_ctl = nullptr;
        kmeans_destroy(ctx);
        return alloc_fail(nullptr);
    }
    for (auto &e : ctx->chunk_ev)
        if (!hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "kmeans_init: hipEventCreate")) {
            e = nullptr;
            kmeans_destroy(ctx);
            return KM_ERR_HIP;
        }
    if (hipHostMalloc((void **)&ctx->host_stat, (NSTAT + 1) * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
        ctx->host_stat = nullptr;
        kmeans_destroy(ctx);
        return alloc_fail(nullptr);
    }
    bool ok = hip_ok(hipMemsetAsync(ctx->a, 0xff, n * sizeof(int32_t), st), "hipMemsetAsync") &&
              hip_ok(hipMemsetAsync(ctx->cerr, 0, sizeof(float), st), "hipMemsetAsync") &&
              hip_ok(hipMemsetAsync(ctx->acc, 0, (size_t)k * ctx->d * 2 * sizeof(int64_t), st), "hipMemsetAsync") &&
              hip_ok(hipMemsetAsync(ctx->cnt, 0, k * sizeof(int32_t), st), "hipMemsetAsync") &&
              hip_ok(hipMemsetAsync(ctx->fin_ticket, 0, sizeof(int32_t), st), "hipMemsetAsync") &&
              hip_ok(hipStreamSynchronize(st), "kmeans_init: hipStreamSynchronize");
    if (!ok) {
        kmeans_destroy(ctx);
        return KM_ERR_HIP;
    }
    // kmeans_run's chunk of steps, captured now so that no run pays for it
    // (a context that records phase times launches its steps one by one)
    if (capture_chunk && !(cfg->flags & KM_FLAG_TIMING))
        (void)chunk_graph(ctx, ctx->c_run);
    if (cfg->workspace_limit_bytes > 0 && ctx_device_bytes(ctx) > (size_t)cfg->workspace_limit_bytes) {
        const size_t used = ctx_device_bytes(ctx);
        kmeans_destroy(ctx);
        if (!cfg->leaf_size && f < MAX_LEAF) // the model's estimate was short: the next coarser index
            return init_context(out, cfg, points, B, pt_off, c_off, stream, capture_chunk, 2 * f);
        set_error("kmeans_init: workspace of " + std::to_string(used) + " bytes exceeds workspace_limit_bytes");
        return KM_ERR_OOM;
    }
    *out = ctx;
    return KM_OK;
}

km_status kmeans_init(km_ctx **out, const km_config *cfg, const void *points, int64_t n, int64_t k, void *stream)
{
    if (!out) {
        set_error("kmeans_init: null output pointer");
        return KM_ERR_INVALID;
    }
    *out = nullptr;
    km_status s = check_config(cfg, n, k);
    if (s != KM_OK)
        return s;
    if (!points) {
        set_error("kmeans_init: null points");
        return KM_ERR_INVALID;
    }
    const int64_t pt_off[2] = {0, n}, c_off[2] = {0, k};
    return init_context(out, cfg, points, 1, pt_off, c_off, stream);
}

// Checks of a batched call's arguments (before any GPU work).
static km_status check_batch(const km_config *cfg, const void *points, const int64_t *pt_offs,
                             const int64_t *c_offs, int32_t B)
{
    if (!cfg || !points || !pt_offs || !c_offs) {
        set_error("batched: null argument");
        return KM_ERR_INVALID;
    }
    if (B < 1) {
        set_error("batched: B must be >= 1");
        return KM_ERR_INVALID;
    }
    if (pt_offs[0] != 0 || c_offs[0] != 0) {
        set_error("batched: pt_offs[0] and c_offs[0] must be 0");
        return KM_ERR_INVALID;
    }
    for (int b = 0; b < B; ++b) {
        const int64_t nb = pt_offs[b + 1] - pt_offs[b], kb = c_offs[b + 1] - c_offs[b];
        if (nb < 1 || kb < 1 || kb > nb) {
            set_error("batched: cloud " + std::to_string(b) + " needs 1 <= k_b <= n_b (got n_b = " +
                      std::to_string(nb) + ", k_b = " + std::to_string(kb) + ")");
            return KM_ERR_INVALID;
        }
        if (B > 1 && kb > TREE_SMALL_K) {
            set_error("batched: cloud " + std::to_string(b) + " has more than " + std::to_string(TREE_SMALL_K) +
                      " centroids (one workgroup builds each cloud's tree)");
            return KM_ERR_UNSUPPORTED;
        }
    }
    km_status s = check_config(cfg, pt_offs[B], c_offs[B]);
    if (s != KM_OK)
        return s;
    if (B > 1 && cfg->algo != KM_INDEXED) {
        set_error("batched: several clouds need KM_INDEXED");
        return KM_ERR_UNSUPPORTED;
    }
    return KM_OK;
}

km_status kmeans_init_batched(km_ctx **out, const km_config *cfg, const void *points, const int64_t *pt_offs,
                              const int64_t *c_offs, int32_t B, void *stream)
{
    if (!out) {
        set_error("kmeans_init_batched: null output pointer");
        return KM_ERR_INVALID;
    }
    *out = nullptr;
    km_status s = check_batch(cfg, points, pt_offs, c_offs, B);
    if (s != KM_OK)
        return s;
    return init_context(out, cfg, points, B, pt_offs, c_offs, stream);
}

km_status kmeans_step(km_ctx *ctx, const double *c_in, double *c_out, int32_t *assign_out, km_iter_stats *stats)
{
    if (!ctx || !c_in || !c_out) {
        set_error("kmeans_step: null argument");
        return KM_ERR_INVALID;
    }
    km_status s = timed_step(ctx, c_in, c_out, assign_out, ctx->steps_done);
    if (s != KM_OK)
        return s;
    ctx->steps_done++;
    if (stats) {
        if (!hip_ok(hipMemcpyAsync(ctx->host_stat, ctx->stat_out, NSTAT * sizeof(int64_t), hipMemcpyDeviceToHost,
                                   ctx->stream),
                    "kmeans_step: stats copy") ||
            !hip_ok(hipMemcpyAsync(ctx->host_stat + NSTAT, ctx->sse_out, sizeof(double), hipMemcpyDeviceToHost,
                                   ctx->stream),
                    "kmeans_step: stats copy") ||
            !hip_ok(hipStreamSynchronize(ctx->stream), "kmeans_step: hipStreamSynchronize"))
            return KM_ERR_HIP;
        fill_stats(ctx, ctx->host_stat, stats);
    }
    return KM_OK;
}

km_status kmeans_run(km_ctx *ctx, double *c_inout, int32_t *assign_out, int32_t max_iter, int32_t stop_when_stable,
                     int32_t *iters_done, km_iter_stats *per_iter)
{
    if (!ctx || !c_inout) {
        set_error("kmeans_run: null argument");
        return KM_ERR_INVALID;
    }
    if (max_iter < 0) {
        set_error("kmeans_run: max_iter must be >= 0");
        return KM_ERR_INVALID;
    }
    hipStream_t st = ctx->stream;
    if (per_iter && ctx->hist_cap < max_iter) { // per-step statistics rows on the device
        if (!hip_ok(hipStreamSynchronize(st), "kmeans_run: hipStreamSynchronize"))
            return KM_ERR_HIP;
        if (ctx->stat_hist)
            (void)hipFree(ctx->stat_hist);
        ctx->stat_hist = nullptr;
        ctx->hist_cap = 0;
        if (ctx->chunk_exec) { // the captured steps write the old rows
            (void)hipGraphExecDestroy(ctx->chunk_exec);
            ctx->chunk_exec = nullptr;
        }
        if (hipMalloc((void **)&ctx->stat_hist, (size_t)max_iter * (NSTAT + 1) * sizeof(int64_t)) != hipSuccess) {
            ctx->stat_hist = nullptr;
            set_error("kmeans_run: device allocation failed");
            return KM_ERR_OOM;
        }
        ctx->hist_cap = max_iter;
    }
    // The steps are launched in chunks without waiting for them; the device
    // counts them and stops the run (every later kernel returns at once)
    // after max_iter steps or at the first stable step.  When the run may
    // stop early, a copy of the control block is taken after every chunk and
    // the host looks at the copy of a chunk only once RUN_AHEAD later chunks
    // are queued, so the device never waits for the host; at most RUN_AHEAD
    // chunks of steps that return at once follow the end of the run.
    km_status s = set_ctl(ctx, max_iter, stop_when_stable ? 1 : 0, 0);
    double *c = ctx->c_run;
    const size_t c_bytes = (size_t)ctx->k * ctx->d * sizeof(double);
    if (s == KM_OK && !hip_ok(hipMemcpyAsync(c, c_inout, c_bytes, hipMemcpyDeviceToDevice, st), "kmeans_run: copy"))
        s = KM_ERR_HIP;
    const bool timing = (ctx->cfg.flags & KM_FLAG_TIMING) != 0;
    int queued = 0; // chunks whose control copies are not yet looked at
    int nchunk = 0;
    for (int launched = 0; s == KM_OK && launched < max_iter;) {
        const int chunk = max_iter - launched < RUN_CHUNK ? max_iter - launched : RUN_CHUNK;
        if (!timing && chunk == RUN_CHUNK && chunk_graph(ctx, c)) {
            if (!hip_ok(hipGraphLaunch(ctx->chunk_exec, st), "kmeans_run: hipGraphLaunch"))
                s = KM_ERR_HIP;
        } else {
            for (int i = 0; s == KM_OK && i < chunk; ++i)
                s = timed_step(ctx, c, c, nullptr, (int64_t)ctx->steps_done + launched + i);
        }
        launched += chunk;
        if (s != KM_OK || !stop_when_stable || launched >= max_iter)
            continue;
        const int slot = nchunk % RUN_AHEAD;
        if (queued == RUN_AHEAD) { // the oldest copy in the ring is about to be reused: look at it
            if (!hip_ok(hipEventSynchronize(ctx->chunk_ev[slot]), "kmeans_run: hipEventSynchronize")) {
                s = KM_ERR_HIP;
                continue;
            }
            --queued;
            if (ctx->host_ctl[slot * CTL_N + CTL_STOP])
                break;
        }
        if (!hip_ok(hipMemcpyAsync(ctx->host_ctl + slot * CTL_N, ctx->ctl, CTL_N * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, st),
                    "kmeans_run: control copy") ||
            !hip_ok(hipEventRecord(ctx->chunk_ev[slot], st), "kmeans_run: hipEventRecord")) {
            s = KM_ERR_HIP;
            continue;
        }
        ++queued;
        ++nchunk;
    }
    if (s != KM_OK) {
        (void)set_ctl(ctx, 0, 0, 1);
        return s;
    }
    int32_t *final_ctl = ctx->host_ctl + RUN_AHEAD * CTL_N;
    if (!hip_ok(hipMemcpyAsync(c_inout, c, c_bytes, hipMemcpyDeviceToDevice, st), "kmeans_run: copy") ||
        !hip_ok(hipMemcpyAsync(final_ctl, ctx->ctl, CTL_N * sizeof(int32_t), hipMemcpyDeviceToHost, st),
                "kmeans_run: control copy") ||
        !hip_ok(hipStreamSynchronize(st), "kmeans_run: hipStreamSynchronize"))
        return KM_ERR_HIP;
    const int32_t iters = final_ctl[CTL_RUN_ITERS];
    if ((s = set_ctl(ctx, 0, 0, 1)) != KM_OK) // back to single steps
        return s;
    ctx->steps_done += iters;
    if (per_iter && iters > 0) {
        std::vector<int64_t> rows((size_t)iters * (NSTAT + 1));
        if (!hip_ok(hipMemcpy(rows.data(), ctx->stat_hist, rows.size() * sizeof(int64_t), hipMemcpyDeviceToHost),
                    "kmeans_run: statistics copy"))
            return KM_ERR_HIP;
        for (int t = 0; t < iters; ++t)
            fill_stats(ctx, rows.data() + (size_t)t * (NSTAT + 1), &per_iter[t]);
    }
    if (assign_out && ctx->steps_done > 0 && (s = scatter_assignment(ctx, assign_out)) != KM_OK)
        return s;
    if (iters_done)
        *iters_done = iters;
    return KM_OK;
}

// A fixed-length run of `iters` steps captured into one graph and launched
// once (the device loop control still counts the steps).  Returns false,
// having launched nothing, if the steps cannot be captured; otherwise s is
// the run's status.
static bool run_captured(km_ctx *ctx, double *c_inout, int32_t *assign_out, int32_t iters, km_status &s)
{
    if (iters == 0 || (ctx->cfg.flags & KM_FLAG_TIMING))
        return false;
    if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        ctx->cap_stream = nullptr;
        (void)hipGetLastError();
        return false;
    }
    hipStream_t st = ctx->stream;
    hipStream_t saved = ctx->stream;
    ctx->stream = ctx->cap_stream;
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    bool ok = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        for (int i = 0; ok && i < iters; ++i)
            ok = step_body(ctx, ctx->c_run, ctx->c_run, nullptr, nullptr, i) == KM_OK;
        ok = hipStreamEndCapture(ctx->cap_stream, &g) == hipSuccess && ok && g;
    }
    ctx->stream = saved;
    if (ok)
        ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
    if (g)
        (void)hipGraphDestroy(g);
    if (!ok) {
        (void)hipGetLastError();
        return false;
    }
    const size_t c_bytes = (size_t)ctx->k * ctx->d * sizeof(double);
    s = set_ctl(ctx, iters, 0, 0);
    if (s == KM_OK &&
        (!hip_ok(hipMemcpyAsync(ctx->c_run, c_inout, c_bytes, hipMemcpyDeviceToDevice, st), "run: copy") ||
         !hip_ok(hipGraphLaunch(ex, st), "run: hipGraphLaunch") ||
         !hip_ok(hipMemcpyAsync(c_inout, ctx->c_run, c_bytes, hipMemcpyDeviceToDevice, st), "run: copy") ||
         !hip_ok(hipStreamSynchronize(st), "run: hipStreamSynchronize")))
        s = KM_ERR_HIP;
    (void)hipGraphExecDestroy(ex);
    if (s == KM_OK)
        s = set_ctl(ctx, 0, 0, 1);
    if (s == KM_OK) {
        ctx->steps_done += iters;
        if (assign_out)
            s = scatter_assignment(ctx, assign_out);
    }
    return true;
}

// Leaf size and leaves per candidate list for a batched run (f, G): the
// given ones, or the fastest of the candidates over 3 timed iterations
// (after one warm-up iteration) on up to 64 evenly spaced clouds.  Cached
// per GPU architecture and workload class.
static km_status autotune(const km_config *cfg, const void *points, const int64_t *pt_offs, const double *c,
                          const int64_t *c_offs, int B, hipStream_t st, int &f_out, int &G_out)
{
    std::vector<int> fs, Gs;
    if (cfg->leaf_size)
        fs.push_back(cfg->leaf_size);
    else
        fs = {16, 32, 64};
    if (cfg->cand_tile)
        Gs.push_back(cfg->cand_tile);
    else
        Gs = {4, 6, 8};
    f_out = fs[0];
    G_out = Gs[0];
    if (fs.size() * Gs.size() == 1)
        return KM_OK;
    static std::mutex mu;
    static std::map<std::string, std::pair<int, int>> cache;
    int dev = 0;
    hipDeviceProp_t prop;
    if (!hip_ok(hipGetDevice(&dev), "autotune: hipGetDevice") ||
        !hip_ok(hipGetDeviceProperties(&prop, dev), "autotune: hipGetDeviceProperties"))
        return KM_ERR_HIP;
    auto lg = [](double v) { return (int)std::lround(std::log2(v > 1.0 ? v : 1.0)); };
    const std::string key = std::string(prop.gcnArchName) + "/d" + std::to_string(cfg->d) + "/n" +
                            std::to_string(lg((double)pt_offs[B] / B)) + "/k" +
                            std::to_string(lg((double)c_offs[B] / B)) + "/f" + std::to_string(cfg->leaf_size) +
                            "/t" + std::to_string(cfg->cand_tile) +
                            ((cfg->flags & KM_FLAG_CELL_LEAVES) ? "/cells" : "") + "/m" +
                            std::to_string(cfg->workspace_limit_bytes);
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            f_out = it->second.first;
            G_out = it->second.second;
            return KM_OK;
        }
    }
    // the sample: clouds floor(i B / S), copied into their own arrays; at
    // least 64 clouds and an eighth of them, so that the candidates' run
    // times are not buried under the fixed cost of each launch
    const int S = B <= 64 ? B : (B / 8 > 64 ? B / 8 : 64);
    const int d = cfg->d;
    std::vector<int64_t> spt(S + 1, 0), sco(S + 1, 0);
    std::vector<int> pick(S);
    for (int i = 0; i < S; ++i) {
        pick[i] = (int)((int64_t)i * B / S);
        spt[i + 1] = spt[i] + (pt_offs[pick[i] + 1] - pt_offs[pick[i]]);
        sco[i + 1] = sco[i] + (c_offs[pick[i] + 1] - c_offs[pick[i]]);
    }
    float *pts = nullptr;
    double *cs = nullptr, *ct = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    km_status s = KM_OK;
    if (hipMalloc((void **)&pts, (size_t)spt[S] * d * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&cs, (size_t)sco[S] * d * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&ct, (size_t)sco[S] * d * sizeof(double)) != hipSuccess) {
        set_error("autotune: device allocation failed");
        s = KM_ERR_OOM;
    }
    if (s == KM_OK && (!hip_ok(hipEventCreate(&e0), "autotune: hipEventCreate") ||
                       !hip_ok(hipEventCreate(&e1), "autotune: hipEventCreate")))
        s = KM_ERR_HIP;
    for (int i = 0; s == KM_OK && i < S; ++i) {
        const int b = pick[i];
        if (!hip_ok(hipMemcpyAsync(pts + spt[i] * d, (const float *)points + pt_offs[b] * d,
                                   (size_t)(pt_offs[b + 1] - pt_offs[b]) * d * sizeof(float), hipMemcpyDeviceToDevice,
                                   st),
                    "autotune: copy") ||
            !hip_ok(hipMemcpyAsync(cs + sco[i] * d, c + c_offs[b] * d,
                                   (size_t)(c_offs[b + 1] - c_offs[b]) * d * sizeof(double), hipMemcpyDeviceToDevice,
                                   st),
                    "autotune: copy"))
            s = KM_ERR_HIP;
    }
    float best = INFINITY;
    bool any = false;
    for (size_t a = 0; s == KM_OK && a < fs.size(); ++a)
        for (size_t g = 0; s == KM_OK && g < Gs.size(); ++g) {
            km_config c2 = *cfg;
            if (cfg->workspace_limit_bytes > 0) { // only candidates whose full-size workspace fits
                c2.leaf_size = fs[a];
                c2.cand_tile = Gs[g];
                if (model_bytes(&c2, B, pt_offs, c_offs, fs[a], Gs[g]) > (size_t)cfg->workspace_limit_bytes)
                    continue;
            }
            any = true;
            c2.leaf_size = fs[a];
            c2.cand_tile = Gs[g];
            c2.flags &= ~(KM_FLAG_TIMING | KM_FLAG_SSE | KM_FLAG_SMALL_LISTS);
            c2.workspace_limit_bytes = 0;
            km_ctx *ctx = nullptr;
            if ((s = init_context(&ctx, &c2, pts, S, spt.data(), sco.data(), st)) != KM_OK)
                break;
            float ms = 0.0f;
            if (!hip_ok(hipMemcpyAsync(ct, cs, (size_t)sco[S] * d * sizeof(double), hipMemcpyDeviceToDevice, st),
                        "autotune: copy") ||
                (s = kmeans_run(ctx, ct, nullptr, 1, 0, nullptr, nullptr)) != KM_OK ||
                !hip_ok(hipEventRecord(e0, st), "autotune: hipEventRecord") ||
                (s = kmeans_run(ctx, ct, nullptr, RUN_CHUNK, 0, nullptr, nullptr)) != KM_OK ||
                !hip_ok(hipEventRecord(e1, st), "autotune: hipEventRecord") ||
                !hip_ok(hipEventSynchronize(e1), "autotune: hipEventSynchronize") ||
                !hip_ok(hipEventElapsedTime(&ms, e0, e1), "autotune: hipEventElapsedTime"))
                s = s == KM_OK ? KM_ERR_HIP : s;
            kmeans_destroy(ctx);
            if (s == KM_OK && ms < best) {
                best = ms;
                f_out = fs[a];
                G_out = Gs[g];
            }
        }
    if (s == KM_OK && !any) {
        set_error("kmeans_run_batched: no leaf size / list length fits workspace_limit_bytes");
        s = KM_ERR_OOM;
    }
    if (e0)
        hipEventDestroy(e0);
    if (e1)
        hipEventDestroy(e1);
    if (pts)
        hipFree(pts);
    if (cs)
        hipFree(cs);
    if (ct)
        hipFree(ct);
    if (s == KM_OK) {
        std::lock_guard<std::mutex> lock(mu);
        cache[key] = {f_out, G_out};
    }
    return s;
}

km_status kmeans_run_batched(const void *points, const int64_t *pt_offs, double *c_inout, const int64_t *c_offs,
                             int32_t *assign_out, int32_t B, const km_config *cfg, int32_t iters, void *stream,
                             int32_t *tuned_out)
{
    km_status s = check_batch(cfg, points, pt_offs, c_offs, B);
    if (s != KM_OK)
        return s;
    if (!c_inout || iters < 0) {
        set_error("kmeans_run_batched: null c_inout or iters < 0");
        return KM_ERR_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    km_config c2 = *cfg;
    if (cfg->algo == KM_INDEXED) {
        int f = 0, G = 0;
        if ((s = autotune(cfg, points, pt_offs, c_inout, c_offs, B, st, f, G)) != KM_OK)
            return s;
        c2.leaf_size = f;
        c2.cand_tile = G;
    }
    km_ctx *ctx = nullptr;
    if ((s = init_context(&ctx, &c2, points, B, pt_offs, c_offs, stream, false)) != KM_OK)
        return s;
    if (!run_captured(ctx, c_inout, assign_out, iters, s)) // capture not possible: the same steps in chunks
        s = kmeans_run(ctx, c_inout, assign_out, iters, 0, nullptr, nullptr);
    if (s == KM_OK && !hip_ok(hipStreamSynchronize(st), "kmeans_run_batched: hipStreamSynchronize"))
        s = KM_ERR_HIP;
    if (s == KM_OK && tuned_out) {
        tuned_out[0] = ctx->f;
        tuned_out[1] = ctx->G;
    }
    kmeans_destroy(ctx);
    return s;
}

} // extern "C"
