// bhq_api.cpp -- the C ABI declared in include/bhq.h: context, validation,
// device memory, uploads, launch and results.  Every failure is reported
// through a return code and a per-context message; nothing aborts.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "bhq.h"
#include "bhq_internal.h"
#include "split_table.h"

using bhq::DevArray;

namespace {

thread_local std::string g_create_error;

enum Arr {
    A_IOFF, A_JPOFF, A_JCOFF, A_ORDER, A_GCX, A_GCY, A_GCZ,
    A_XI, A_YI, A_ZI, A_E2I,
    A_JPX, A_JPY, A_JPZ, A_JPM,
    A_JCX, A_JCY, A_JCZ, A_JCM, A_Q00, A_Q01, A_Q02, A_Q11, A_Q12, A_Q22,
    A_JCT,
    A_AX, A_AY, A_AZ, A_POT,
    A_QUEUE,
    A_POOLP, A_POOLC, A_JPIDX, A_JCIDX,
    A_TORDER, A_ENERGY, A_OSCRATCH, A_SORTSCRATCH, A_PART, A_FLAG, A_LIVE, A_CLOCK,
    A_COUNT
};

bool finite_all(const double *v, int64_t n)
{
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return false;
    return true;
}

// Slot table of a group dispatch order (see bhq_plan_order).  Offsets are
// already validated.  Throws std::bad_alloc.
std::vector<int32_t> plan_order(int64_t ng, const int64_t *i_off,
                                const int64_t *jp_off, const int64_t *jc_off,
                                int mode, int window, int tail, int xcds)
{
    std::vector<uint64_t> cost((size_t)ng);
    for (int64_t g = 0; g < ng; ++g)
        cost[(size_t)g] = bhq::order_cost(i_off[g + 1] - i_off[g], jp_off[g + 1] - jp_off[g],
                                          jc_off[g + 1] - jc_off[g]);
    auto costly_first = [&](int32_t a, int32_t b) {
        return cost[(size_t)a] > cost[(size_t)b];
    };
    if (mode == BHQ_ORDER_COST) {
        std::vector<int32_t> order((size_t)ng);
        for (int64_t g = 0; g < ng; ++g) order[(size_t)g] = (int32_t)g;
        std::stable_sort(order.begin(), order.end(), costly_first);
        return order;
    }
    // contiguous pieces of equal cost: group g goes to the piece holding the
    // midpoint of its cost interval (monotone in g)
    uint64_t total = 0;
    for (uint64_t c : cost) total += c;
    std::vector<std::vector<int32_t>> piece((size_t)xcds);
    uint64_t before = 0;
    for (int64_t g = 0; g < ng; ++g) {
        const int x = bhq::order_piece(before, cost[(size_t)g], total, xcds, g, ng);
        before += cost[(size_t)g];
        piece[(size_t)x].push_back((int32_t)g);
    }
    // windows of `window` groups from the start of a piece, and its last
    // `tail` groups as one more window; each sorted costly first
    // (pieces are independent: one host thread each when there is work)
    auto sort_piece = [&](std::vector<int32_t> &pc) {
        const size_t n = pc.size();
        const size_t body = n > (size_t)tail ? n - (size_t)tail : 0;
        for (size_t w = 0; w < body; w += (size_t)window) {
            const size_t e = std::min(body, w + (size_t)window);
            std::stable_sort(pc.begin() + (ptrdiff_t)w, pc.begin() + (ptrdiff_t)e,
                             costly_first);
        }
        std::stable_sort(pc.begin() + (ptrdiff_t)body, pc.end(), costly_first);
    };
    if (ng >= (int64_t)1 << 16) {
        std::vector<std::thread> pool;
        try {
            for (auto &pc : piece) pool.emplace_back(sort_piece, std::ref(pc));
        } catch (const std::system_error &) {
            // no threads: the pieces not started are sorted below
        }
        for (auto &t : pool) t.join();
        for (size_t x = pool.size(); x < piece.size(); ++x) sort_piece(piece[x]);
    } else {
        for (auto &pc : piece) sort_piece(pc);
    }
    size_t longest = 0;
    for (auto &pc : piece) longest = std::max(longest, pc.size());
    std::vector<int32_t> order(longest * (size_t)xcds, -1);
    for (int x = 0; x < xcds; ++x)
        for (size_t k = 0; k < piece[(size_t)x].size(); ++k)
            order[k * (size_t)xcds + (size_t)x] = piece[(size_t)x][k];
    return order;
}

bool valid_order(int mode, int window, int tail)
{
    return (mode == BHQ_ORDER_COST || mode == BHQ_ORDER_XCD) && window >= 1 &&
           window <= (1 << 24) && tail >= 0 && tail <= (1 << 24);
}

}  // namespace

struct bhq_ctx {
    int device = 0;
    int kernel = BHQ_QUAD;
    int precision = BHQ_FP32_OFS64;
    std::string err;

    int64_t ng = -1, ni = 0, njp = 0, njc = 0;
    // Host copies of the group offsets.  After a device build they are
    // copied from the device arrays on first use (off_stale).
    std::vector<int64_t> i_off, jp_off, jc_off;
    bool off_stale = false;
    DevArray arr[A_COUNT];

    bool have_i = false, have_jp = false, have_jc = false, have_t = false;
    // list mode after bhq_set_groups: 0 undecided, 1 materialised, 2 indexed
    int list_mode = 0;
    // > 0: index lists in per-group slots of these sizes (a rebuilt
    // device list); 0: compact lists at the offsets
    int64_t list_slot_p = 0, list_slot_c = 0;
    int64_t npool_p = -1, npool_c = -1;
    // The particle pool is in tree order and A_TORDER[k] is the input index
    // of pool entry k (lists from bhq_set_lists_indexed or
    // bhq_build_lists_device).
    bool tree_order = false;
    DevArray tbuf[bhq::T_COUNT_];  // device list builder working memory
    bool have_jp_idx = false, have_jc_idx = false;
    int eps_mode = 0;  // 0 none, 1 uniform, 2 per-particle
    double eps2_all = 0.0;
    bool have_split = false;
    double rs = 0.0, rcut = 0.0, box = 0.0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool launched = false;
    int clock_khz = 0;                  // bhq_clock_begin: constant counter rate
    hipStream_t clock_stream = nullptr;
    hipStream_t last_stream = nullptr;

    bhq::LaunchCfg cfg;
    int use_graph = 0;
    int order_mode = BHQ_ORDER_XCD, order_window = BHQ_ORDER_WINDOW,
        order_tail = BHQ_ORDER_TAIL;
    int64_t nslots = 0;
    // device builds: slot sizes for the next one-walk build, and what the
    // last build did (one walk or not, longest particle and cell lists)
    int64_t walk_cap_p = 0, walk_cap_c = 0;
    // depth and cell count of the last device-built tree
    int tree_levels = 0;
    int64_t tree_cells = 0;
    int64_t build_info[3] = {0, 0, 0};
    uint64_t args_version = 0;  // bumped when device pointers/params change
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    struct {
        int kernel, precision, block, i_per_thread, persistent, blocks_per_cu, jsplit,
            waves_per_eu;
        uint64_t version;
    } graph_key{};

    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
    }

    std::vector<double> stage;  // host staging for SoA transposes

    int fail(int code, const char *fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    int hip_fail(hipError_t e, const char *what)
    {
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            return fail(BHQ_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
        return fail(BHQ_E_HIP, "%s: %s", what, hipGetErrorString(e));
    }
    int select()
    {
        hipError_t e = hipSetDevice(device);
        return e == hipSuccess ? BHQ_OK : hip_fail(e, "hipSetDevice");
    }
    // Wait until the last compute has finished with the inputs (it may run
    // on a stream that does not synchronise with the null stream, which the
    // host uploads use).
    void quiesce()
    {
        if (launched) (void)hipEventSynchronize(ev1);
    }
    // Upload n doubles to array a at element offset off.
    int put(Arr a, int64_t off, const double *src, int64_t n)
    {
        if (n == 0) return BHQ_OK;
        quiesce();
        hipError_t e = hipMemcpy(arr[a].as<double>() + off, src,
                                 (size_t)n * sizeof(double),
                                 hipMemcpyHostToDevice);
        return e == hipSuccess ? BHQ_OK : hip_fail(e, "hipMemcpy H2D");
    }
    // Upload component c of an AoS array v[n][w] into array a at offset off.
    int put_component(Arr a, int64_t off, const double *v, int w, int c,
                      int64_t n)
    {
        try {
            stage.resize((size_t)n);
        } catch (const std::bad_alloc &) {
            return fail(BHQ_E_NOMEM, "host staging of %lld values",
                        (long long)n);
        }
        for (int64_t k = 0; k < n; ++k) stage[(size_t)k] = v[k * w + c];
        return put(a, off, stage.data(), n);
    }
    // Allocate the materialised list arrays (first set_jp / set_jc after
    // set_groups).
    int use_materialised()
    {
        if (list_mode == 2)
            return fail(BHQ_E_STATE, "lists already given as indices since "
                                     "the last set_groups");
        if (list_mode == 1) return BHQ_OK;
        quiesce();
        const size_t D = sizeof(double);
        const Arr jp[] = {A_JPX, A_JPY, A_JPZ, A_JPM};
        const Arr jc[] = {A_JCX, A_JCY, A_JCZ, A_JCM, A_Q00, A_Q01, A_Q02,
                          A_Q11, A_Q12, A_Q22, A_JCT};
        for (Arr a : jp) {
            hipError_t e = arr[a].reserve((size_t)njp * D);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        }
        for (Arr a : jc) {
            hipError_t e = arr[a].reserve((size_t)njc * D);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        }
        list_mode = 1;
        ++args_version;
        return BHQ_OK;
    }
    int use_indexed()
    {
        if (list_mode == 1)
            return fail(BHQ_E_STATE, "lists already materialised since the "
                                     "last set_groups");
        if (list_mode == 2) return BHQ_OK;
        quiesce();
        hipError_t e = arr[A_JPIDX].reserve((size_t)njp * 4);
        if (e == hipSuccess) e = arr[A_JCIDX].reserve((size_t)njc * 4);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        list_mode = 2;
        ++args_version;
        return BHQ_OK;
    }
    // Make the host copies of the offsets current (after a device build the
    // device arrays are complete when the build returns).
    int host_offsets()
    {
        if (!off_stale) return BHQ_OK;
        const int rc = select();
        if (rc != BHQ_OK) return rc;
        try {
            for (auto *v : {&i_off, &jp_off, &jc_off}) v->resize((size_t)ng + 1);
        } catch (const std::bad_alloc &) {
            return fail(BHQ_E_NOMEM, "host copy of offsets");
        }
        const struct {
            Arr a;
            std::vector<int64_t> *v;
        } cp[3] = {{A_IOFF, &i_off}, {A_JPOFF, &jp_off}, {A_JCOFF, &jc_off}};
        for (const auto &c : cp) {
            hipError_t e = hipMemcpy(c.v->data(), arr[c.a].p, ((size_t)ng + 1) * 8,
                                     hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "offsets D2H");
        }
        off_stale = false;
        return BHQ_OK;
    }
    // Compute the slot table for the current groups and order mode and
    // upload it.
    int upload_order()
    {
        const int rc = host_offsets();
        if (rc != BHQ_OK) return rc;
        std::vector<int32_t> order;
        try {
            order = plan_order(ng, i_off.data(), jp_off.data(), jc_off.data(),
                               order_mode, order_window, order_tail, BHQ_XCDS);
        } catch (const std::bad_alloc &) {
            return fail(BHQ_E_NOMEM, "host order table");
        }
        if (launched) (void)hipEventSynchronize(ev1);
        hipError_t e = arr[A_ORDER].reserve(order.size() * 4);
        if (e == hipSuccess)
            e = hipMemcpy(arr[A_ORDER].p, order.data(), order.size() * 4,
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "order upload");
        nslots = (int64_t)order.size();
        ++args_version;
        return BHQ_OK;
    }
    // Turn lists kept in per-group slots into compact lists at the offsets
    // (before entries are written at compact addresses).  Waits for all
    // work on the device first: a launch in flight may still read them.
    int unslot_lists()
    {
        const struct {
            Arr a, off;
            int64_t *slot, cnt;
        } lists[2] = {{A_JPIDX, A_JPOFF, &list_slot_p, njp}, {A_JCIDX, A_JCOFF, &list_slot_c, njc}};
        for (const auto &l : lists) {
            if (*l.slot <= 0) continue;
            hipError_t e = hipDeviceSynchronize();
            if (e == hipSuccess) e = arr[A_SORTSCRATCH].reserve((size_t)std::max<int64_t>(l.cnt, 1) * 4);
            if (e == hipSuccess)
                e = bhq::launch_compact_lists(ng, arr[l.off].as<int64_t>(), arr[l.a].as<int32_t>(),
                                              *l.slot, arr[A_SORTSCRATCH].as<int32_t>(), nullptr);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "list compaction");
            std::swap(arr[l.a], arr[A_SORTSCRATCH]);
            *l.slot = 0;
            ++args_version;
        }
        return BHQ_OK;
    }
    // Copy a compact index list (cnt entries, group offsets in device array
    // off) to the host; lists kept in per-group slots of `slot` entries are
    // compacted on the device first, into the scratch array (after all work
    // on the device, which may still use that array, has finished).
    int fetch_list(Arr a, Arr off, int64_t slot, int64_t cnt, int32_t *dst)
    {
        const void *src = arr[a].p;
        hipError_t e = hipSuccess;
        if (slot > 0) {
            e = hipDeviceSynchronize();
            if (e == hipSuccess) e = arr[A_SORTSCRATCH].reserve((size_t)cnt * 4);
            if (e == hipSuccess)
                e = bhq::launch_compact_lists(ng, arr[off].as<int64_t>(), arr[a].as<int32_t>(),
                                              slot, arr[A_SORTSCRATCH].as<int32_t>(), nullptr);
            src = arr[A_SORTSCRATCH].p;
        }
        if (e == hipSuccess) e = hipMemcpy(dst, src, (size_t)cnt * 4, hipMemcpyDeviceToHost);
        return e == hipSuccess ? BHQ_OK : hip_fail(e, "list copy");
    }
    // Every i-particle's eps^2 = eps2_all, filled on the device (stream s,
    // synchronised: the forces may be computed on another stream).
    int fill_eps_uniform(hipStream_t s = nullptr)
    {
        if (ni == 0) return BHQ_OK;
        if (launched) (void)hipEventSynchronize(ev1);
        hipError_t e = bhq::launch_fill_f64(arr[A_E2I].as<double>(), ni, eps2_all, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e == hipSuccess ? BHQ_OK : hip_fail(e, "eps fill");
    }
};

#define CHECK_CTX(ctx)                                    \
    do {                                                  \
        if (!(ctx)) return BHQ_E_ARG;                     \
    } while (0)

#define TRY(expr)                                         \
    do {                                                  \
        int rc_ = (expr);                                 \
        if (rc_ != BHQ_OK) return rc_;                    \
    } while (0)

static bool valid_kernel(int k) { return k >= BHQ_MONO && k <= BHQ_QUAD_SOFT; }
static bool valid_prec(int p) { return p == BHQ_FP32_OFS64 || p == BHQ_FP64; }

extern "C" {

int bhq_create(bhq_ctx **out, int device, int kernel, int precision)
{
    if (!out) {
        g_create_error = "bhq_create: out is NULL";
        return BHQ_E_ARG;
    }
    *out = nullptr;
    if (!valid_kernel(kernel) || !valid_prec(precision)) {
        g_create_error = "bhq_create: unknown kernel or precision";
        return BHQ_E_ARG;
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        g_create_error = std::string("bhq_create: no GPU available (") +
                         hipGetErrorString(e) + ")";
        return BHQ_E_NODEV;
    }
    if (device < 0 || device >= count) {
        g_create_error = "bhq_create: device index out of range";
        return BHQ_E_NODEV;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_create_error = std::string("bhq_create: hipSetDevice: ") +
                         hipGetErrorString(e);
        return BHQ_E_HIP;
    }
    bhq_ctx *c = new (std::nothrow) bhq_ctx();
    if (!c) {
        g_create_error = "bhq_create: out of host memory";
        return BHQ_E_NOMEM;
    }
    c->device = device;
    c->kernel = kernel;
    c->precision = precision;
    if (hipDeviceGetAttribute(&c->cfg.num_cu, hipDeviceAttributeMultiprocessorCount,
                              device) != hipSuccess ||
        c->cfg.num_cu <= 0 || c->arr[A_QUEUE].reserve(256) != hipSuccess) {
        g_create_error = "bhq_create: device query or allocation failed";
        c->arr[A_QUEUE].release();
        delete c;
        return BHQ_E_HIP;
    }
    // the static working memory of bhq_compute_noalloc: find its address
    // on this device once (device current)
    if (bhq::scratch_init(device) != hipSuccess) {
        g_create_error = "bhq_create: static working memory not found on the device";
        c->arr[A_QUEUE].release();
        delete c;
        return BHQ_E_HIP;
    }
    if (hipEventCreate(&c->ev0) != hipSuccess ||
        hipEventCreate(&c->ev1) != hipSuccess) {
        g_create_error = "bhq_create: hipEventCreate failed";
        if (c->ev0) (void)hipEventDestroy(c->ev0);
        c->arr[A_QUEUE].release();
        delete c;
        return BHQ_E_HIP;
    }
    g_create_error.clear();
    *out = c;
    return BHQ_OK;
}

int bhq_destroy(bhq_ctx *ctx)
{
    if (!ctx) return BHQ_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->launched) (void)hipEventSynchronize(ctx->ev1);
    ctx->drop_graph();
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto &a : ctx->arr) a.release();
    for (auto &a : ctx->tbuf) a.release();
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
    return BHQ_OK;
}

int bhq_set_kernel(bhq_ctx *ctx, int kernel, int precision)
{
    CHECK_CTX(ctx);
    if (!valid_kernel(kernel) || !valid_prec(precision))
        return ctx->fail(BHQ_E_ARG, "bhq_set_kernel: unknown kernel %d or "
                                    "precision %d", kernel, precision);
    ctx->kernel = kernel;
    ctx->precision = precision;
    return BHQ_OK;
}

int bhq_set_eps(bhq_ctx *ctx, double eps)
{
    CHECK_CTX(ctx);
    if (!std::isfinite(eps)) return ctx->fail(BHQ_E_NONFINITE, "eps not finite");
    if (!(eps > 0.0) || !(eps * eps >= bhq::kMinEps2))
        return ctx->fail(BHQ_E_ARG, "eps^2 must be >= 2^-126 (a normal FP32 number): the "
                                    "softened kernels include each particle's self pair");
    ctx->eps2_all = eps * eps;
    ctx->eps_mode = 1;
    if (ctx->ng >= 0) {
        TRY(ctx->select());
        return ctx->fill_eps_uniform();
    }
    return BHQ_OK;
}

int bhq_set_eps2_i(bhq_ctx *ctx, int64_t ni, const double *eps2)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "set_eps2_i before set_groups");
    if (!eps2 && ni > 0) return ctx->fail(BHQ_E_ARG, "eps2 is NULL");
    if (ni != ctx->ni)
        return ctx->fail(BHQ_E_RANGE, "set_eps2_i: ni %lld != %lld",
                         (long long)ni, (long long)ctx->ni);
    for (int64_t k = 0; k < ni; ++k) {
        if (!std::isfinite(eps2[k]))
            return ctx->fail(BHQ_E_NONFINITE, "eps2[%lld] not finite",
                             (long long)k);
        if (!(eps2[k] >= bhq::kMinEps2))
            return ctx->fail(BHQ_E_ARG, "eps2[%lld] must be >= 2^-126 (the softened "
                             "kernels include the self pair)", (long long)k);
    }
    TRY(ctx->select());
    TRY(ctx->put(A_E2I, 0, eps2, ni));
    ctx->eps_mode = 2;
    return BHQ_OK;
}

int bhq_set_split(bhq_ctx *ctx, double rs, double rcut, double box)
{
    CHECK_CTX(ctx);
    if (!std::isfinite(rs) || !std::isfinite(rcut) || !std::isfinite(box))
        return ctx->fail(BHQ_E_NONFINITE, "split parameters not finite");
    if (!(rs > 0.0) || !(rcut > 0.0) || box < 0.0)
        return ctx->fail(BHQ_E_ARG, "need rs > 0, rcut > 0, box >= 0");
    ctx->rs = rs;
    ctx->rcut = rcut;
    ctx->box = box;
    ctx->have_split = true;
    ++ctx->args_version;
    return BHQ_OK;
}

static int check_offsets(bhq_ctx *ctx, const char *name, const int64_t *off,
                         int64_t ng)
{
    if (!off) return ctx->fail(BHQ_E_ARG, "%s is NULL", name);
    if (off[0] != 0) return ctx->fail(BHQ_E_RANGE, "%s[0] != 0", name);
    for (int64_t g = 0; g < ng; ++g)
        if (off[g + 1] < off[g])
            return ctx->fail(BHQ_E_RANGE, "%s not monotone at group %lld", name,
                             (long long)g);
    return BHQ_OK;
}

int bhq_set_groups(bhq_ctx *ctx, int64_t ng, const int64_t *i_off,
                   const double (*center)[3], const int64_t *jp_off,
                   const int64_t *jc_off)
{
    CHECK_CTX(ctx);
    if (ng < 1) return ctx->fail(BHQ_E_ARG, "ng must be >= 1");
    if (ng > 0x7fffffff) return ctx->fail(BHQ_E_RANGE, "too many groups");
    if (!center) return ctx->fail(BHQ_E_ARG, "center is NULL");
    TRY(check_offsets(ctx, "i_off", i_off, ng));
    TRY(check_offsets(ctx, "jp_off", jp_off, ng));
    TRY(check_offsets(ctx, "jc_off", jc_off, ng));
    if (!finite_all(&center[0][0], 3 * ng))
        return ctx->fail(BHQ_E_NONFINITE, "group centre not finite");
    TRY(ctx->select());

    const int64_t ni = i_off[ng], njp = jp_off[ng], njc = jc_off[ng];
    const size_t D = sizeof(double);
    struct { Arr a; size_t bytes; } need[] = {
        {A_IOFF, (size_t)(ng + 1) * 8}, {A_JPOFF, (size_t)(ng + 1) * 8},
        {A_JCOFF, (size_t)(ng + 1) * 8},
        {A_GCX, (size_t)ng * D}, {A_GCY, (size_t)ng * D}, {A_GCZ, (size_t)ng * D},
        {A_XI, (size_t)ni * D}, {A_YI, (size_t)ni * D}, {A_ZI, (size_t)ni * D},
        {A_E2I, (size_t)ni * D},
        {A_AX, (size_t)ni * D}, {A_AY, (size_t)ni * D}, {A_AZ, (size_t)ni * D},
        {A_POT, (size_t)ni * D},
    };
    if (ctx->launched) (void)hipEventSynchronize(ctx->ev1);
    for (auto &n : need) {
        hipError_t e = ctx->arr[n.a].reserve(n.bytes);
        if (e != hipSuccess) {
            ctx->ng = -1;
            return ctx->hip_fail(e, "hipMalloc");
        }
    }
    try {
        ctx->i_off.assign(i_off, i_off + ng + 1);
        ctx->jp_off.assign(jp_off, jp_off + ng + 1);
        ctx->jc_off.assign(jc_off, jc_off + ng + 1);
        ctx->off_stale = false;
    } catch (const std::bad_alloc &) {
        ctx->ng = -1;
        return ctx->fail(BHQ_E_NOMEM, "host copy of offsets");
    }
    ctx->ng = ng;
    ctx->ni = ni;
    ctx->njp = njp;
    ctx->njc = njc;
    ++ctx->args_version;
    ctx->have_i = ctx->have_jp = ctx->have_jc = ctx->have_t = false;
    ctx->have_jp_idx = ctx->have_jc_idx = false;
    ctx->list_mode = 0;
    ctx->list_slot_p = ctx->list_slot_c = 0;
    ctx->tree_order = false;
    if (ctx->eps_mode == 2) ctx->eps_mode = 0;

    auto up = [&](Arr a, const void *src, size_t bytes) -> int {
        if (!bytes) return BHQ_OK;
        hipError_t e = hipMemcpy(ctx->arr[a].p, src, bytes, hipMemcpyHostToDevice);
        return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, "hipMemcpy H2D");
    };
    TRY(up(A_IOFF, i_off, (size_t)(ng + 1) * 8));
    TRY(up(A_JPOFF, jp_off, (size_t)(ng + 1) * 8));
    TRY(up(A_JCOFF, jc_off, (size_t)(ng + 1) * 8));
    for (int c = 0; c < 3; ++c)
        TRY(ctx->put_component((Arr)(A_GCX + c), 0, &center[0][0], 3, c, ng));

    ctx->nslots = 0;
    const int rc = ctx->upload_order();
    if (rc != BHQ_OK) {
        ctx->ng = -1;
        return rc;
    }
    if (ctx->eps_mode == 1) TRY(ctx->fill_eps_uniform());
    return BHQ_OK;
}

int bhq_set_i(bhq_ctx *ctx, int64_t ni, const double (*x)[3])
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "set_i before set_groups");
    if (ni != ctx->ni)
        return ctx->fail(BHQ_E_RANGE, "set_i: ni %lld != i_off[ng] %lld",
                         (long long)ni, (long long)ctx->ni);
    if (!x && ni > 0) return ctx->fail(BHQ_E_ARG, "x is NULL");
    if (!finite_all(&x[0][0], 3 * ni))
        return ctx->fail(BHQ_E_NONFINITE, "i position not finite");
    TRY(ctx->select());
    for (int c = 0; c < 3; ++c)
        TRY(ctx->put_component((Arr)(A_XI + c), 0, &x[0][0], 3, c, ni));
    ctx->have_i = true;
    return BHQ_OK;
}

int bhq_set_jp(bhq_ctx *ctx, int64_t adr, int64_t n, const double (*x)[3],
               const double *m)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "set_jp before set_groups");
    if (adr < 0 || n < 0) return ctx->fail(BHQ_E_ARG, "negative adr or n");
    if (adr + n > ctx->njp)
        return ctx->fail(BHQ_E_RANGE, "set_jp: adr + n = %lld > njp = %lld",
                         (long long)(adr + n), (long long)ctx->njp);
    if (n > 0 && (!x || !m)) return ctx->fail(BHQ_E_ARG, "x or m is NULL");
    if (!finite_all(&x[0][0], 3 * n) || !finite_all(m, n))
        return ctx->fail(BHQ_E_NONFINITE, "j-particle data not finite");
    TRY(ctx->select());
    TRY(ctx->use_materialised());
    for (int c = 0; c < 3; ++c)
        TRY(ctx->put_component((Arr)(A_JPX + c), adr, &x[0][0], 3, c, n));
    TRY(ctx->put(A_JPM, adr, m, n));
    ctx->have_jp = true;
    return BHQ_OK;
}

int bhq_set_jc(bhq_ctx *ctx, int64_t adr, int64_t n, const double (*x)[3],
               const double *m, const double (*q)[6], const double *trace)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "set_jc before set_groups");
    if (adr < 0 || n < 0) return ctx->fail(BHQ_E_ARG, "negative adr or n");
    if (adr + n > ctx->njc)
        return ctx->fail(BHQ_E_RANGE, "set_jc: adr + n = %lld > njc = %lld",
                         (long long)(adr + n), (long long)ctx->njc);
    if (n > 0 && (!x || !m || !q))
        return ctx->fail(BHQ_E_ARG, "x, m or q is NULL");
    if (!finite_all(&x[0][0], 3 * n) || !finite_all(m, n) ||
        !finite_all(&q[0][0], 6 * n) || (trace && !finite_all(trace, n)))
        return ctx->fail(BHQ_E_NONFINITE, "j-cell data not finite");
    TRY(ctx->select());
    TRY(ctx->use_materialised());
    for (int c = 0; c < 3; ++c)
        TRY(ctx->put_component((Arr)(A_JCX + c), adr, &x[0][0], 3, c, n));
    TRY(ctx->put(A_JCM, adr, m, n));
    for (int c = 0; c < 6; ++c)
        TRY(ctx->put_component((Arr)(A_Q00 + c), adr, &q[0][0], 6, c, n));
    if (trace) {
        TRY(ctx->put(A_JCT, adr, trace, n));
    } else if (n > 0) {
        try {
            ctx->stage.assign((size_t)n, 0.0);
        } catch (const std::bad_alloc &) {
            return ctx->fail(BHQ_E_NOMEM, "host staging");
        }
        TRY(ctx->put(A_JCT, adr, ctx->stage.data(), n));
    }
    ctx->have_jc = true;
    return BHQ_OK;
}

// Checks that a compute can run and fills the kernel arguments from the
// context (results into the context's arrays).
static int prepare_compute(bhq_ctx *ctx, bhq::ForceArgs &A)
{
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "compute before set_groups");
    if (!ctx->have_i && ctx->ni > 0)
        return ctx->fail(BHQ_E_STATE, "compute before set_i");
    if (ctx->list_mode == 2) {
        if (ctx->njp > 0 && !ctx->have_jp_idx)
            return ctx->fail(BHQ_E_STATE, "compute before set_jp_idx");
        if (ctx->njc > 0 && !ctx->have_jc_idx)
            return ctx->fail(BHQ_E_STATE, "compute before set_jc_idx");
    } else {
        if (ctx->njp > 0 && !ctx->have_jp)
            return ctx->fail(BHQ_E_STATE, "compute before set_jp");
        if (ctx->njc > 0 && !ctx->have_jc)
            return ctx->fail(BHQ_E_STATE, "compute before set_jc");
        if (ctx->njp + ctx->njc > 0 && ctx->list_mode != 1)
            return ctx->fail(BHQ_E_STATE, "compute before the lists are set");
    }
    const bool split = ctx->kernel == BHQ_SPLIT_QUAD ||
                       ctx->kernel == BHQ_SPLIT_MONO;
    if (split && !ctx->have_split)
        return ctx->fail(BHQ_E_STATE, "split kernel without bhq_set_split");
    if (split && ctx->precision == BHQ_FP32_OFS64 &&
        ctx->rcut > 2.0 * (double)bhq::kSplitDomain * ctx->rs)
        return ctx->fail(BHQ_E_ARG, "FP32 split kernels need rcut <= %g rs "
                         "(the range of their erfc evaluation); use BHQ_FP64",
                         2.0 * (double)bhq::kSplitDomain);
    if (!split && ctx->eps_mode == 0)
        return ctx->fail(BHQ_E_STATE, "compute before set_eps / set_eps2_i");
    TRY(ctx->select());

    A = bhq::ForceArgs{};
    auto D = [&](Arr a) { return ctx->arr[a].as<double>(); };
    A.ng = ctx->ng;
    A.nslots = ctx->nslots;
    A.order = ctx->arr[A_ORDER].as<int32_t>();
    A.xcds = ctx->order_mode == BHQ_ORDER_XCD ? BHQ_XCDS : 0;
    A.i_off = ctx->arr[A_IOFF].as<int64_t>();
    A.jp_off = ctx->arr[A_JPOFF].as<int64_t>();
    A.jc_off = ctx->arr[A_JCOFF].as<int64_t>();
    A.gcx = D(A_GCX); A.gcy = D(A_GCY); A.gcz = D(A_GCZ);
    A.xi = D(A_XI); A.yi = D(A_YI); A.zi = D(A_ZI); A.e2i = D(A_E2I);
    A.jpx = D(A_JPX); A.jpy = D(A_JPY); A.jpz = D(A_JPZ); A.jpm = D(A_JPM);
    A.jcx = D(A_JCX); A.jcy = D(A_JCY); A.jcz = D(A_JCZ); A.jcm = D(A_JCM);
    A.q00 = D(A_Q00); A.q01 = D(A_Q01); A.q02 = D(A_Q02);
    A.q11 = D(A_Q11); A.q12 = D(A_Q12); A.q22 = D(A_Q22);
    A.jct = D(A_JCT);
    A.ax = D(A_AX); A.ay = D(A_AY); A.az = D(A_AZ); A.pot = D(A_POT);
    A.out_stride = 1;
    A.ni = ctx->ni;
    A.box = split ? ctx->box : 0.0;
    A.rs = ctx->rs;
    A.rcut = ctx->rcut;

    A.queue = ctx->arr[A_QUEUE].as<unsigned int>();
    if (ctx->list_mode == 2) {
        A.pool_p = ctx->arr[A_POOLP].as<bhq::PartRec>();
        A.pool_c = ctx->arr[A_POOLC].as<bhq::CellRec>();
        A.jp_idx = ctx->arr[A_JPIDX].as<int32_t>();
        A.jc_idx = ctx->arr[A_JCIDX].as<int32_t>();
        A.jp_slot = ctx->list_slot_p;
        A.jc_slot = ctx->list_slot_c;
    }

    return BHQ_OK;
}

int bhq_compute(bhq_ctx *ctx, void *stream)
{
    CHECK_CTX(ctx);
    bhq::ForceArgs A;
    TRY(prepare_compute(ctx, A));

    if (ctx->cfg.jsplit > 1) {
        // parts of every i-particle's sums (32 B per entry covers FP64)
        const size_t bytes = (size_t)ctx->cfg.jsplit * (size_t)ctx->ni * 32;
        if (bytes > ctx->arr[A_PART].cap) {
            ctx->quiesce();
            hipError_t e = ctx->arr[A_PART].reserve(bytes);
            if (e != hipSuccess) return ctx->hip_fail(e, "hipMalloc (j-split parts)");
            ++ctx->args_version;
        }
        A.part = ctx->arr[A_PART].p;
    }

    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (ctx->use_graph) {
        const bool same =
            ctx->graph_exec && ctx->graph_key.kernel == ctx->kernel &&
            ctx->graph_key.precision == ctx->precision &&
            ctx->graph_key.block == ctx->cfg.block &&
            ctx->graph_key.i_per_thread == ctx->cfg.i_per_thread &&
            ctx->graph_key.persistent == ctx->cfg.persistent &&
            ctx->graph_key.blocks_per_cu == ctx->cfg.blocks_per_cu &&
            ctx->graph_key.jsplit == ctx->cfg.jsplit &&
            ctx->graph_key.waves_per_eu == ctx->cfg.waves_per_eu &&
            ctx->graph_key.version == ctx->args_version;
        if (!same) {
            if (ctx->launched) (void)hipEventSynchronize(ctx->ev1);
            ctx->drop_graph();
            if (!ctx->cap_stream) {
                e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
                if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamCreate");
            }
            e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamBeginCapture");
            const hipError_t le =
                bhq::launch_force(ctx->kernel, ctx->precision, A, ctx->cfg,
                                  ctx->cap_stream);
            e = hipStreamEndCapture(ctx->cap_stream, &ctx->graph);
            if (le != hipSuccess) {
                ctx->drop_graph();
                return ctx->hip_fail(le, "force kernel capture");
            }
            if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&ctx->graph_exec, ctx->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                ctx->drop_graph();
                return ctx->hip_fail(e, "hipGraphInstantiate");
            }
            ctx->graph_key.kernel = ctx->kernel;
            ctx->graph_key.precision = ctx->precision;
            ctx->graph_key.block = ctx->cfg.block;
            ctx->graph_key.i_per_thread = ctx->cfg.i_per_thread;
            ctx->graph_key.persistent = ctx->cfg.persistent;
            ctx->graph_key.blocks_per_cu = ctx->cfg.blocks_per_cu;
            ctx->graph_key.jsplit = ctx->cfg.jsplit;
            ctx->graph_key.waves_per_eu = ctx->cfg.waves_per_eu;
            ctx->graph_key.version = ctx->args_version;
        }
        e = hipEventRecord(ctx->ev0, s);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipEventRecord");
        e = hipGraphLaunch(ctx->graph_exec, s);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipGraphLaunch");
    } else {
        e = hipEventRecord(ctx->ev0, s);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipEventRecord");
        e = bhq::launch_force(ctx->kernel, ctx->precision, A, ctx->cfg, s);
        if (e != hipSuccess) return ctx->hip_fail(e, "force kernel launch");
    }
    e = hipEventRecord(ctx->ev1, s);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventRecord");
    ctx->launched = true;
    ctx->last_stream = s;
    return BHQ_OK;
}

static int check_device_range(bhq_ctx *ctx, const void *p, size_t bytes, const char *name);

int bhq_compute_noalloc(bhq_ctx *ctx, double *a, double *pot, void *stream)
{
    CHECK_CTX(ctx);
    if (!a) return ctx->fail(BHQ_E_ARG, "compute_noalloc: a is NULL");
    bhq::ForceArgs A;
    TRY(prepare_compute(ctx, A));
    const size_t entry = ctx->precision == BHQ_FP64 ? 32 : 16;
    if (ctx->cfg.jsplit > 1 &&
        (size_t)ctx->cfg.jsplit * (size_t)ctx->ni * entry > bhq::kScratchPartBytes)
        return ctx->fail(BHQ_E_RANGE,
                         "compute_noalloc: jsplit %d x %lld i-particles x %zu B of parts "
                         "exceed the static %zu B (use a smaller jsplit, or bhq_compute)",
                         ctx->cfg.jsplit, (long long)ctx->ni, entry, bhq::kScratchPartBytes);
    if (ctx->ni > 0) {
        TRY(check_device_range(ctx, a, (size_t)ctx->ni * 3 * sizeof(double), "a"));
        if (pot) TRY(check_device_range(ctx, pot, (size_t)ctx->ni * sizeof(double), "pot"));
    }
    char *sp = static_cast<char *>(bhq::scratch_ptr(ctx->device));
    if (!sp) return ctx->fail(BHQ_E_STATE, "compute_noalloc: static working memory not found");
    A.ax = a;
    A.ay = a + 1;
    A.az = a + 2;
    A.pot = pot;
    A.out_stride = 3;
    A.queue = reinterpret_cast<unsigned int *>(sp);
    A.part = sp + bhq::kScratchQueueBytes;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipEventRecord(ctx->ev0, s);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventRecord");
    e = bhq::launch_force(ctx->kernel, ctx->precision, A, ctx->cfg, s);
    if (e != hipSuccess) return ctx->hip_fail(e, "force kernel launch");
    e = hipEventRecord(ctx->ev1, s);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventRecord");
    ctx->launched = true;
    ctx->last_stream = s;
    return BHQ_OK;
}

int bhq_count_live(bhq_ctx *ctx, int64_t *pp, int64_t *pc)
{
    CHECK_CTX(ctx);
    if (!pp || !pc) return ctx->fail(BHQ_E_ARG, "count_live: NULL output");
    if (ctx->kernel != BHQ_SPLIT_QUAD && ctx->kernel != BHQ_SPLIT_MONO)
        return ctx->fail(BHQ_E_STATE, "count_live: the context's kernel has no cutoff");
    bhq::ForceArgs A;
    TRY(prepare_compute(ctx, A));
    ctx->quiesce();
    hipError_t e = ctx->arr[A_LIVE].reserve(256);
    unsigned long long h[2] = {0, 0};
    auto *d = ctx->arr[A_LIVE].as<unsigned long long>();
    if (e == hipSuccess) e = hipMemcpy(d, h, sizeof(h), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = bhq::launch_count_live(A, d, nullptr);
    if (e == hipSuccess) e = hipMemcpy(h, d, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ctx->hip_fail(e, "count_live");
    *pp = (int64_t)h[0];
    *pc = (int64_t)h[1];
    return BHQ_OK;
}

int bhq_clock_begin(bhq_ctx *ctx, double wall_ms, void *stream)
{
    CHECK_CTX(ctx);
    if (!(wall_ms > 0.0) || !(wall_ms <= 10000.0))
        return ctx->fail(BHQ_E_ARG, "clock_begin: wall_ms must be in (0, 10000]");
    TRY(ctx->select());
    int khz = 0;
    hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device);
    if (e == hipSuccess && khz <= 0) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = ctx->arr[A_CLOCK].reserve(256);
    if (e == hipSuccess)
        e = bhq::launch_clock_window((unsigned long long)(wall_ms * (double)khz),
                                     ctx->arr[A_CLOCK].as<unsigned long long>(),
                                     static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return ctx->hip_fail(e, "clock_begin");
    ctx->clock_khz = khz;
    ctx->clock_stream = static_cast<hipStream_t>(stream);
    return BHQ_OK;
}

int bhq_clock_end(bhq_ctx *ctx, double *mhz)
{
    CHECK_CTX(ctx);
    if (!mhz) return ctx->fail(BHQ_E_ARG, "clock_end: NULL output");
    if (ctx->clock_khz <= 0) return ctx->fail(BHQ_E_STATE, "clock_end before clock_begin");
    TRY(ctx->select());
    unsigned long long h[4] = {0, 0, 0, 0};
    hipError_t e = hipStreamSynchronize(ctx->clock_stream);
    if (e == hipSuccess)
        e = hipMemcpy(h, ctx->arr[A_CLOCK].p, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ctx->hip_fail(e, "clock_end");
    if (h[3] <= h[1]) return ctx->fail(BHQ_E_STATE, "clock_end: empty window");
    *mhz = (double)(h[2] - h[0]) / (double)(h[3] - h[1]) * (double)ctx->clock_khz * 1e-3;
    ctx->clock_khz = 0;
    return BHQ_OK;
}

int bhq_set_tuning(bhq_ctx *ctx, int block, int i_per_thread, int blocks_per_cu,
                   int persistent, int use_graph, int jsplit, int waves_per_eu)
{
    CHECK_CTX(ctx);
    if (block == 0) block = 256;
    if (i_per_thread == 0) i_per_thread = 2;
    if (jsplit == 0) jsplit = 1;
    if (jsplit != 1 && jsplit != 2 && jsplit != 4 && jsplit != 8)
        return ctx->fail(BHQ_E_ARG, "jsplit must be 1, 2, 4 or 8 (or 0)");
    if (block != 128 && block != 256)
        return ctx->fail(BHQ_E_ARG, "block must be 128 or 256 (or 0)");
    if (i_per_thread != 1 && i_per_thread != 2)
        return ctx->fail(BHQ_E_ARG, "i_per_thread must be 1 or 2 (or 0)");
    if (blocks_per_cu < 0 || blocks_per_cu > 64)
        return ctx->fail(BHQ_E_ARG, "blocks_per_cu must be in [0, 64]");
    if ((persistent != 0 && persistent != 1) || (use_graph != 0 && use_graph != 1))
        return ctx->fail(BHQ_E_ARG, "persistent and use_graph are 0 or 1");
    if (waves_per_eu != 0 && waves_per_eu != 6 && waves_per_eu != 8)
        return ctx->fail(BHQ_E_ARG, "waves_per_eu must be 0, 6 or 8");
    if (waves_per_eu != 0 && block != 256)
        return ctx->fail(BHQ_E_ARG, "waves_per_eu 6 and 8 exist for block 256 only");
    ctx->cfg.block = block;
    ctx->cfg.waves_per_eu = waves_per_eu;
    ctx->cfg.i_per_thread = i_per_thread;
    ctx->cfg.blocks_per_cu = blocks_per_cu;
    ctx->cfg.persistent = persistent;
    ctx->cfg.jsplit = jsplit;
    ctx->use_graph = use_graph;
    return BHQ_OK;
}

int bhq_get_tuning(const bhq_ctx *ctx, int out[7])
{
    if (!ctx || !out) return BHQ_E_ARG;
    out[0] = ctx->cfg.block;
    out[1] = ctx->cfg.i_per_thread;
    out[2] = ctx->cfg.blocks_per_cu;
    out[3] = ctx->cfg.persistent;
    out[4] = ctx->use_graph;
    out[5] = ctx->cfg.jsplit;
    out[6] = ctx->cfg.waves_per_eu;
    return BHQ_OK;
}

int bhq_set_group_order(bhq_ctx *ctx, int mode, int window, int tail)
{
    CHECK_CTX(ctx);
    if (!valid_order(mode, window, tail))
        return ctx->fail(BHQ_E_ARG, "group order: mode %d window %d tail %d "
                         "(mode 0 or 1, window in [1, 2^24], tail in [0, 2^24])",
                         mode, window, tail);
    ctx->order_mode = mode;
    ctx->order_window = window;
    ctx->order_tail = tail;
    if (ctx->ng < 0) return BHQ_OK;
    TRY(ctx->select());
    const int rc = ctx->upload_order();
    if (rc != BHQ_OK) ctx->ng = -1;  // no valid order table: set_groups again
    return rc;
}

int bhq_get_group_order(const bhq_ctx *ctx, int out[3])
{
    if (!ctx || !out) return BHQ_E_ARG;
    out[0] = ctx->order_mode;
    out[1] = ctx->order_window;
    out[2] = ctx->order_tail;
    return BHQ_OK;
}

int bhq_get_build_info(const bhq_ctx *ctx, int64_t out[3])
{
    CHECK_CTX(ctx);
    if (!out) return BHQ_E_ARG;
    for (int k = 0; k < 3; ++k) out[k] = ctx->build_info[k];
    return BHQ_OK;
}

int bhq_get_order(bhq_ctx *ctx, int32_t *order, int64_t cap, int64_t *nslots)
{
    CHECK_CTX(ctx);
    if (!nslots) return ctx->fail(BHQ_E_ARG, "get_order: null nslots");
    if (ctx->ng < 0 || ctx->nslots <= 0) return ctx->fail(BHQ_E_STATE, "get_order: no groups");
    *nslots = ctx->nslots;
    if (!order) return BHQ_OK;
    if (cap < ctx->nslots) return ctx->fail(BHQ_E_RANGE, "get_order: cap too small");
    TRY(ctx->select());
    if (ctx->launched) (void)hipEventSynchronize(ctx->ev1);
    hipError_t e = hipMemcpy(order, ctx->arr[A_ORDER].p, (size_t)ctx->nslots * 4,
                             hipMemcpyDeviceToHost);
    return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, "order copy");
}

int bhq_plan_order(int64_t ng, const int64_t *i_off, const int64_t *jp_off,
                   const int64_t *jc_off, int mode, int window, int tail,
                   int xcds, int32_t *order, int64_t cap, int64_t *nslots)
{
    if (ng < 1 || ng > 0x7fffffff || !i_off || !jp_off || !jc_off || !nslots)
        return BHQ_E_ARG;
    if (!valid_order(mode, window, tail) || xcds < 1 || xcds > bhq::kQueueWords)
        return BHQ_E_ARG;
    for (const int64_t *off : {i_off, jp_off, jc_off}) {
        if (off[0] != 0) return BHQ_E_RANGE;
        for (int64_t g = 0; g < ng; ++g)
            if (off[g + 1] < off[g]) return BHQ_E_RANGE;
    }
    std::vector<int32_t> o;
    try {
        o = plan_order(ng, i_off, jp_off, jc_off, mode, window, tail, xcds);
    } catch (const std::bad_alloc &) {
        return BHQ_E_NOMEM;
    }
    *nslots = (int64_t)o.size();
    if (!order) return BHQ_OK;
    if (cap < (int64_t)o.size()) return BHQ_E_RANGE;
    std::copy(o.begin(), o.end(), order);
    return BHQ_OK;
}

int bhq_set_pool_particles(bhq_ctx *ctx, int64_t n, const double (*x)[3],
                           const double *m)
{
    CHECK_CTX(ctx);
    if (n < 0 || n > 0x7fffffffLL) return ctx->fail(BHQ_E_ARG, "bad pool size");
    if (n > 0 && (!x || !m)) return ctx->fail(BHQ_E_ARG, "x or m is NULL");
    if (n > 0 && (!finite_all(&x[0][0], 3 * n) || !finite_all(m, n)))
        return ctx->fail(BHQ_E_NONFINITE, "particle pool not finite");
    TRY(ctx->select());
    std::vector<bhq::PartRec> rec;
    try {
        rec.resize((size_t)n);
    } catch (const std::bad_alloc &) {
        return ctx->fail(BHQ_E_NOMEM, "host staging");
    }
    for (int64_t k = 0; k < n; ++k)
        rec[(size_t)k] = bhq::PartRec{x[k][0], x[k][1], x[k][2], m[k]};
    ctx->quiesce();
    hipError_t e = ctx->arr[A_POOLP].reserve((size_t)n * sizeof(bhq::PartRec));
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(ctx->arr[A_POOLP].p, rec.data(),
                      (size_t)n * sizeof(bhq::PartRec), hipMemcpyHostToDevice);
    if (e != hipSuccess) return ctx->hip_fail(e, "particle pool upload");
    ctx->npool_p = n;
    ctx->tree_order = false;
    ctx->have_jp_idx = false;  // indices are validated against the pool
    ++ctx->args_version;
    return BHQ_OK;
}

int bhq_set_pool_cells(bhq_ctx *ctx, int64_t n, const double (*x)[3],
                       const double *m, const double (*q)[6],
                       const double *trace)
{
    CHECK_CTX(ctx);
    if (n < 0 || n > 0x7fffffffLL) return ctx->fail(BHQ_E_ARG, "bad pool size");
    if (n > 0 && (!x || !m || !q)) return ctx->fail(BHQ_E_ARG, "x, m or q is NULL");
    if (n > 0 && (!finite_all(&x[0][0], 3 * n) || !finite_all(m, n) ||
                  !finite_all(&q[0][0], 6 * n) || (trace && !finite_all(trace, n))))
        return ctx->fail(BHQ_E_NONFINITE, "cell pool not finite");
    TRY(ctx->select());
    std::vector<bhq::CellRec> rec;
    try {
        rec.resize((size_t)n);
    } catch (const std::bad_alloc &) {
        return ctx->fail(BHQ_E_NOMEM, "host staging");
    }
    for (int64_t k = 0; k < n; ++k)
        rec[(size_t)k] = bhq::CellRec{x[k][0], x[k][1], x[k][2], m[k],
                                      q[k][0], q[k][1], q[k][2], q[k][3],
                                      q[k][4], q[k][5], trace ? trace[k] : 0.0,
                                      0.0};
    ctx->quiesce();
    hipError_t e = ctx->arr[A_POOLC].reserve((size_t)n * sizeof(bhq::CellRec));
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(ctx->arr[A_POOLC].p, rec.data(),
                      (size_t)n * sizeof(bhq::CellRec), hipMemcpyHostToDevice);
    if (e != hipSuccess) return ctx->hip_fail(e, "cell pool upload");
    ctx->npool_c = n;
    ctx->have_jc_idx = false;
    ++ctx->args_version;
    return BHQ_OK;
}

static int set_idx(bhq_ctx *ctx, Arr a, int64_t total, int64_t pool,
                   int64_t adr, int64_t n, const int32_t *idx, const char *what)
{
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "%s before set_groups", what);
    if (pool < 0)
        return ctx->fail(BHQ_E_STATE, "%s before its pool is set", what);
    if (adr < 0 || n < 0) return ctx->fail(BHQ_E_ARG, "negative adr or n");
    if (adr + n > total)
        return ctx->fail(BHQ_E_RANGE, "%s: adr + n = %lld > %lld", what,
                         (long long)(adr + n), (long long)total);
    if (n > 0 && !idx) return ctx->fail(BHQ_E_ARG, "idx is NULL");
    for (int64_t k = 0; k < n; ++k)
        if (idx[k] < 0 || idx[k] >= pool)
            return ctx->fail(BHQ_E_RANGE, "%s: index %d at %lld outside the "
                             "pool of %lld", what, (int)idx[k],
                             (long long)(adr + k), (long long)pool);
    TRY(ctx->select());
    TRY(ctx->use_indexed());
    if (n == 0) return BHQ_OK;
    TRY(ctx->unslot_lists());
    ctx->quiesce();
    hipError_t e = hipMemcpy(ctx->arr[a].as<int32_t>() + adr, idx,
                             (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice);
    return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, "hipMemcpy H2D");
}

int bhq_set_jp_idx(bhq_ctx *ctx, int64_t adr, int64_t n, const int32_t *idx)
{
    CHECK_CTX(ctx);
    TRY(set_idx(ctx, A_JPIDX, ctx->njp, ctx->npool_p, adr, n, idx, "set_jp_idx"));
    ctx->have_jp_idx = true;
    return BHQ_OK;
}

int bhq_set_jc_idx(bhq_ctx *ctx, int64_t adr, int64_t n, const int32_t *idx)
{
    CHECK_CTX(ctx);
    TRY(set_idx(ctx, A_JCIDX, ctx->njc, ctx->npool_c, adr, n, idx, "set_jc_idx"));
    ctx->have_jc_idx = true;
    return BHQ_OK;
}

int bhq_get_result(bhq_ctx *ctx, double (*a)[3], double *pot)
{
    CHECK_CTX(ctx);
    if (!ctx->launched) return ctx->fail(BHQ_E_STATE, "no compute launched");
    TRY(ctx->select());
    hipError_t e = hipEventSynchronize(ctx->ev1);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventSynchronize");
    const int64_t ni = ctx->ni;
    if (ni == 0) return BHQ_OK;
    try {
        ctx->stage.resize((size_t)ni);
    } catch (const std::bad_alloc &) {
        return ctx->fail(BHQ_E_NOMEM, "host staging");
    }
    if (a) {
        for (int c = 0; c < 3; ++c) {
            e = hipMemcpy(ctx->stage.data(), ctx->arr[A_AX + c].p,
                          (size_t)ni * sizeof(double), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return ctx->hip_fail(e, "hipMemcpy D2H");
            for (int64_t k = 0; k < ni; ++k) a[k][c] = ctx->stage[(size_t)k];
        }
    }
    if (pot) {
        e = hipMemcpy(pot, ctx->arr[A_POT].p, (size_t)ni * sizeof(double),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipMemcpy D2H");
    }
    return BHQ_OK;
}

int bhq_get_counts(const bhq_ctx *ctx, int64_t *n_pp, int64_t *n_pc)
{
    if (!ctx || !n_pp || !n_pc) return BHQ_E_ARG;
    if (ctx->ng < 0) return BHQ_E_STATE;
    // the host offsets are a cache of the device arrays: filling it leaves
    // the context's state unchanged
    const int rc = const_cast<bhq_ctx *>(ctx)->host_offsets();
    if (rc != BHQ_OK) return rc;
    int64_t pp = 0, pc = 0;
    for (int64_t g = 0; g < ctx->ng; ++g) {
        const int64_t nig = ctx->i_off[(size_t)g + 1] - ctx->i_off[(size_t)g];
        pp += nig * (ctx->jp_off[(size_t)g + 1] - ctx->jp_off[(size_t)g]);
        pc += nig * (ctx->jc_off[(size_t)g + 1] - ctx->jc_off[(size_t)g]);
    }
    *n_pp = pp;
    *n_pc = pc;
    return BHQ_OK;
}

int bhq_get_kernel_ms(bhq_ctx *ctx, double *ms)
{
    CHECK_CTX(ctx);
    if (!ms) return ctx->fail(BHQ_E_ARG, "ms is NULL");
    if (!ctx->launched) return ctx->fail(BHQ_E_STATE, "no compute launched");
    TRY(ctx->select());
    hipError_t e = hipEventSynchronize(ctx->ev1);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventSynchronize");
    float f = 0.0f;
    e = hipEventElapsedTime(&f, ctx->ev0, ctx->ev1);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventElapsedTime");
    *ms = (double)f;
    return BHQ_OK;
}

const char *bhq_last_error(const bhq_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

// Upload host-built lists: gathers i-particles into group order and
// materialises the j-entries in chunks to bound host memory.
int bhq_set_lists(bhq_ctx *ctx, const bhq_lists *L, const double (*x)[3],
                  const double *m)
{
    CHECK_CTX(ctx);
    if (!L || !x || !m) return ctx->fail(BHQ_E_ARG, "NULL lists, x or m");
    int64_t sz[4];
    TRY(bhq_lists_sizes(L, sz));
    const int64_t ng = sz[0], njp = sz[1], njc = sz[2], ncell = sz[3];
    try {
        std::vector<int64_t> i_off((size_t)ng + 1), jp_off((size_t)ng + 1),
            jc_off((size_t)ng + 1);
        std::vector<double> center((size_t)ng * 3);
        TRY(bhq_lists_export(L, nullptr, i_off.data(),
                             reinterpret_cast<double(*)[3]>(center.data()),
                             nullptr, jp_off.data(), nullptr, jc_off.data(),
                             nullptr));
        TRY(bhq_set_groups(ctx, ng, i_off.data(),
                           reinterpret_cast<const double(*)[3]>(center.data()),
                           jp_off.data(), jc_off.data()));
        const int64_t n = i_off[(size_t)ng];
        {
            std::vector<int64_t> i_idx((size_t)n);
            TRY(bhq_lists_export(L, i_idx.data(), nullptr, nullptr, nullptr,
                                 nullptr, nullptr, nullptr, nullptr));
            std::vector<double> xi((size_t)n * 3);
            for (int64_t k = 0; k < n; ++k)
                for (int c = 0; c < 3; ++c)
                    xi[(size_t)(3 * k + c)] = x[i_idx[(size_t)k]][c];
            TRY(bhq_set_i(ctx, n, reinterpret_cast<const double(*)[3]>(xi.data())));
        }
        const int64_t chunk = 1 << 22;
        {
            std::vector<int64_t> jp_idx((size_t)njp);
            TRY(bhq_lists_export(L, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 jp_idx.data(), nullptr, nullptr));
            std::vector<double> bx, bm;
            for (int64_t a0 = 0; a0 < njp; a0 += chunk) {
                const int64_t cn = std::min(chunk, njp - a0);
                bx.resize((size_t)cn * 3);
                bm.resize((size_t)cn);
                for (int64_t k = 0; k < cn; ++k) {
                    const int64_t p = jp_idx[(size_t)(a0 + k)];
                    for (int c = 0; c < 3; ++c) bx[(size_t)(3 * k + c)] = x[p][c];
                    bm[(size_t)k] = m[p];
                }
                TRY(bhq_set_jp(ctx, a0, cn,
                               reinterpret_cast<const double(*)[3]>(bx.data()),
                               bm.data()));
            }
            if (njp == 0) ctx->have_jp = true;
        }
        {
            std::vector<int32_t> jc_cell((size_t)njc);
            TRY(bhq_lists_export(L, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, jc_cell.data()));
            std::vector<double> com((size_t)ncell * 3), mass((size_t)ncell),
                q((size_t)ncell * 6), tr((size_t)ncell);
            TRY(bhq_lists_cells(L, reinterpret_cast<double(*)[3]>(com.data()),
                                mass.data(),
                                reinterpret_cast<double(*)[6]>(q.data()),
                                tr.data()));
            std::vector<double> bx, bm, bq, bt;
            for (int64_t a0 = 0; a0 < njc; a0 += chunk) {
                const int64_t cn = std::min(chunk, njc - a0);
                bx.resize((size_t)cn * 3);
                bm.resize((size_t)cn);
                bq.resize((size_t)cn * 6);
                bt.resize((size_t)cn);
                for (int64_t k = 0; k < cn; ++k) {
                    const size_t c = (size_t)jc_cell[(size_t)(a0 + k)];
                    for (int d = 0; d < 3; ++d)
                        bx[(size_t)(3 * k + d)] = com[3 * c + d];
                    for (int d = 0; d < 6; ++d)
                        bq[(size_t)(6 * k + d)] = q[6 * c + d];
                    bm[(size_t)k] = mass[c];
                    bt[(size_t)k] = tr[c];
                }
                TRY(bhq_set_jc(ctx, a0, cn,
                               reinterpret_cast<const double(*)[3]>(bx.data()),
                               bm.data(),
                               reinterpret_cast<const double(*)[6]>(bq.data()),
                               bt.data()));
            }
            if (njc == 0) ctx->have_jc = true;
        }
    } catch (const std::bad_alloc &) {
        return ctx->fail(BHQ_E_NOMEM, "host memory while materialising lists");
    }
    return BHQ_OK;
}

// Upload host-built lists as index lists into shared pools: the particles in
// input order, the tree cells, and per-entry int32 indices.
int bhq_set_lists_indexed(bhq_ctx *ctx, const bhq_lists *L,
                          const double (*x)[3], const double *m)
{
    CHECK_CTX(ctx);
    if (!L || !x || !m) return ctx->fail(BHQ_E_ARG, "NULL lists, x or m");
    int64_t sz[4];
    TRY(bhq_lists_sizes(L, sz));
    const int64_t ng = sz[0], njp = sz[1], njc = sz[2], ncell = sz[3];
    try {
        std::vector<int64_t> i_off((size_t)ng + 1), jp_off((size_t)ng + 1),
            jc_off((size_t)ng + 1);
        std::vector<double> center((size_t)ng * 3);
        TRY(bhq_lists_export(L, nullptr, i_off.data(),
                             reinterpret_cast<double(*)[3]>(center.data()),
                             nullptr, jp_off.data(), nullptr, jc_off.data(),
                             nullptr));
        TRY(bhq_set_groups(ctx, ng, i_off.data(),
                           reinterpret_cast<const double(*)[3]>(center.data()),
                           jp_off.data(), jc_off.data()));
        const int64_t n = i_off[(size_t)ng];
        // particles in tree order: pool entry k is input particle i_idx[k]
        std::vector<int64_t> i_idx((size_t)n);
        TRY(bhq_lists_export(L, i_idx.data(), nullptr, nullptr, nullptr,
                             nullptr, nullptr, nullptr, nullptr));
        {
            std::vector<double> xs((size_t)n * 3), ms((size_t)n);
            for (int64_t k = 0; k < n; ++k) {
                for (int c = 0; c < 3; ++c)
                    xs[(size_t)(3 * k + c)] = x[i_idx[(size_t)k]][c];
                ms[(size_t)k] = m[i_idx[(size_t)k]];
            }
            TRY(bhq_set_i(ctx, n, reinterpret_cast<const double(*)[3]>(xs.data())));
            TRY(bhq_set_pool_particles(
                ctx, n, reinterpret_cast<const double(*)[3]>(xs.data()), ms.data()));
        }
        {
            std::vector<double> com((size_t)ncell * 3), mass((size_t)ncell),
                q((size_t)ncell * 6), tr((size_t)ncell);
            TRY(bhq_lists_cells(L, reinterpret_cast<double(*)[3]>(com.data()),
                                mass.data(),
                                reinterpret_cast<double(*)[6]>(q.data()),
                                tr.data()));
            TRY(bhq_set_pool_cells(ctx, ncell,
                                   reinterpret_cast<const double(*)[3]>(com.data()),
                                   mass.data(),
                                   reinterpret_cast<const double(*)[6]>(q.data()),
                                   tr.data()));
        }
        std::vector<int32_t> pos((size_t)n);
        for (int64_t k = 0; k < n; ++k) pos[(size_t)i_idx[(size_t)k]] = (int32_t)k;
        {
            std::vector<int64_t> jp64((size_t)njp);
            TRY(bhq_lists_export(L, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 jp64.data(), nullptr, nullptr));
            std::vector<int32_t> jp32((size_t)njp);
            for (int64_t k = 0; k < njp; ++k) jp32[(size_t)k] = pos[(size_t)jp64[(size_t)k]];
            std::vector<int64_t>().swap(jp64);
            TRY(bhq_set_jp_idx(ctx, 0, njp, jp32.data()));
        }
        {
            std::vector<int32_t> jc((size_t)njc);
            TRY(bhq_lists_export(L, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, jc.data()));
            TRY(bhq_set_jc_idx(ctx, 0, njc, jc.data()));
        }
        {
            std::vector<int32_t> o32((size_t)n);
            for (int64_t k = 0; k < n; ++k) o32[(size_t)k] = (int32_t)i_idx[(size_t)k];
            hipError_t e = ctx->arr[A_TORDER].reserve((size_t)n * 4);
            if (e == hipSuccess)
                e = hipMemcpy(ctx->arr[A_TORDER].p, o32.data(), (size_t)n * 4,
                              hipMemcpyHostToDevice);
            if (e != hipSuccess) return ctx->hip_fail(e, "order upload");
            ctx->tree_order = true;
        }
    } catch (const std::bad_alloc &) {
        return ctx->fail(BHQ_E_NOMEM, "host memory while uploading index lists");
    }
    return BHQ_OK;
}

// Device memory check: [p, p + bytes) inside one device allocation.
static int check_device_range(bhq_ctx *ctx, const void *p, size_t bytes,
                              const char *name)
{
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, const_cast<void *>(p));
    if (e != hipSuccess || !base) {
        (void)hipGetLastError();
        return ctx->fail(BHQ_E_ARG, "%s is not device memory", name);
    }
    const char *b = static_cast<const char *>(base);
    const char *q = static_cast<const char *>(p);
    if (q < b || (size_t)(q - b) + bytes > size)
        return ctx->fail(BHQ_E_RANGE, "%s: %zu bytes do not fit its allocation",
                         name, bytes);
    return BHQ_OK;
}

/* ------------------------------------------------------------------------
 * Set calls that read caller device memory (bhq_set_*_dev).  Each one waits
 * for the context's last compute, validates the caller's arrays on the
 * device, and only then copies them into the context's arrays with device
 * kernels on `stream`; it returns when the copy is complete.
 * ------------------------------------------------------------------------ */

// Run the validation kernels queued by checks(flag) on s, wait for them and
// turn the flag into a return code.
extern "C++" template <typename F>
static int dev_check(bhq_ctx *ctx, hipStream_t s, const char *what, F checks)
{
    hipError_t e = ctx->arr[A_FLAG].reserve(256);
    unsigned *flag = ctx->arr[A_FLAG].as<unsigned>();
    if (e == hipSuccess) e = bhq::launch_clear_flag(flag, s);
    if (e == hipSuccess) e = checks(flag);
    unsigned h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return ctx->hip_fail(e, what);
    if (h & bhq::kBadNonFinite) return ctx->fail(BHQ_E_NONFINITE, "%s: NaN or infinity", what);
    if (h & bhq::kBadNonPositive) return ctx->fail(BHQ_E_ARG, "%s: a value below 2^-126", what);
    if (h & bhq::kBadOrder)
        return ctx->fail(BHQ_E_RANGE, "%s: offsets not starting at 0 or not monotone", what);
    if (h & bhq::kBadRange) return ctx->fail(BHQ_E_RANGE, "%s: index outside the pool", what);
    return BHQ_OK;
}

static int dev_done(bhq_ctx *ctx, hipError_t e, hipStream_t s, const char *what)
{
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, what);
}

int bhq_set_groups_dev(bhq_ctx *ctx, int64_t ng, const int64_t *i_off,
                       const double (*center)[3], const int64_t *jp_off,
                       const int64_t *jc_off, void *stream)
{
    CHECK_CTX(ctx);
    if (ng < 1) return ctx->fail(BHQ_E_ARG, "ng must be >= 1");
    if (ng > 0x7fffffff) return ctx->fail(BHQ_E_RANGE, "too many groups");
    if (!i_off || !center || !jp_off || !jc_off)
        return ctx->fail(BHQ_E_ARG, "set_groups_dev: NULL array");
    TRY(ctx->select());
    const size_t ob = ((size_t)ng + 1) * 8;
    TRY(check_device_range(ctx, i_off, ob, "i_off"));
    TRY(check_device_range(ctx, jp_off, ob, "jp_off"));
    TRY(check_device_range(ctx, jc_off, ob, "jc_off"));
    TRY(check_device_range(ctx, center, (size_t)ng * 24, "center"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->quiesce();
    TRY(dev_check(ctx, s, "set_groups_dev", [&](unsigned *f) {
        hipError_t e = bhq::launch_check_offsets(i_off, ng, f, s);
        if (e == hipSuccess) e = bhq::launch_check_offsets(jp_off, ng, f, s);
        if (e == hipSuccess) e = bhq::launch_check_offsets(jc_off, ng, f, s);
        if (e == hipSuccess) e = bhq::launch_check_f64(&center[0][0], 3 * ng, false, f, s);
        return e;
    }));
    int64_t tot[3] = {0, 0, 0};
    const int64_t *offs[3] = {i_off, jp_off, jc_off};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        e = hipMemcpyAsync(&tot[k], offs[k] + ng, 8, hipMemcpyDeviceToHost, s);
    if ((e = (e == hipSuccess ? hipStreamSynchronize(s) : e)) != hipSuccess)
        return ctx->hip_fail(e, "set_groups_dev: totals");
    const int64_t ni = tot[0], njp = tot[1], njc = tot[2];
    const size_t D = sizeof(double);
    const struct { Arr a; size_t bytes; } need[] = {
        {A_IOFF, ob}, {A_JPOFF, ob}, {A_JCOFF, ob},
        {A_GCX, (size_t)ng * D}, {A_GCY, (size_t)ng * D}, {A_GCZ, (size_t)ng * D},
        {A_XI, (size_t)ni * D}, {A_YI, (size_t)ni * D}, {A_ZI, (size_t)ni * D},
        {A_E2I, (size_t)ni * D},
        {A_AX, (size_t)ni * D}, {A_AY, (size_t)ni * D}, {A_AZ, (size_t)ni * D},
        {A_POT, (size_t)ni * D},
    };
    for (auto &q : need) {
        e = ctx->arr[q.a].reserve(q.bytes);
        if (e != hipSuccess) {
            ctx->ng = -1;
            return ctx->hip_fail(e, "hipMalloc");
        }
    }
    e = hipMemcpyAsync(ctx->arr[A_IOFF].p, i_off, ob, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->arr[A_JPOFF].p, jp_off, ob, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->arr[A_JCOFF].p, jc_off, ob, hipMemcpyDeviceToDevice, s);
    double *gc[3] = {ctx->arr[A_GCX].as<double>(), ctx->arr[A_GCY].as<double>(),
                     ctx->arr[A_GCZ].as<double>()};
    if (e == hipSuccess) e = bhq::launch_unpack(&center[0][0], ng, 3, gc, s);
    if (dev_done(ctx, e, s, "set_groups_dev: copy") != BHQ_OK) {
        ctx->ng = -1;
        return BHQ_E_HIP;
    }
    ctx->ng = ng;
    ctx->ni = ni;
    ctx->njp = njp;
    ctx->njc = njc;
    ctx->off_stale = true;
    ++ctx->args_version;
    ctx->have_i = ctx->have_jp = ctx->have_jc = ctx->have_t = false;
    ctx->have_jp_idx = ctx->have_jc_idx = false;
    ctx->list_mode = 0;
    ctx->list_slot_p = ctx->list_slot_c = 0;
    ctx->tree_order = false;
    if (ctx->eps_mode == 2) ctx->eps_mode = 0;
    ctx->nslots = 0;
    int orc;
    if (ctx->order_mode == BHQ_ORDER_XCD &&
        bhq::plan_order_device_supported(ctx->order_window, ctx->order_tail)) {
        // the offsets are on the device: plan the dispatch order there
        int64_t ns = 0;
        std::string msg;
        orc = bhq::plan_order_device(ng, ctx->arr[A_IOFF].as<int64_t>(),
                                     ctx->arr[A_JPOFF].as<int64_t>(),
                                     ctx->arr[A_JCOFF].as<int64_t>(), ctx->order_window,
                                     ctx->order_tail, BHQ_XCDS, ctx->arr[A_ORDER],
                                     ctx->arr[A_OSCRATCH], &ns, s, &msg);
        if (orc == BHQ_OK)
            ctx->nslots = ns;
        else
            ctx->fail(orc, "%s", msg.c_str());
    } else {
        orc = ctx->upload_order();
    }
    if (orc != BHQ_OK) {
        ctx->ng = -1;
        return orc;
    }
    if (ctx->eps_mode == 1) TRY(ctx->fill_eps_uniform(s));
    return BHQ_OK;
}

int bhq_set_i_dev(bhq_ctx *ctx, int64_t ni, const double (*x)[3], void *stream)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "set_i_dev before set_groups");
    if (ni != ctx->ni)
        return ctx->fail(BHQ_E_RANGE, "set_i_dev: ni %lld != i_off[ng] %lld",
                         (long long)ni, (long long)ctx->ni);
    if (ni == 0) {
        ctx->have_i = true;
        return BHQ_OK;
    }
    if (!x) return ctx->fail(BHQ_E_ARG, "x is NULL");
    TRY(ctx->select());
    TRY(check_device_range(ctx, x, (size_t)ni * 24, "x"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->quiesce();
    TRY(dev_check(ctx, s, "set_i_dev", [&](unsigned *f) {
        return bhq::launch_check_f64(&x[0][0], 3 * ni, false, f, s);
    }));
    double *out[3] = {ctx->arr[A_XI].as<double>(), ctx->arr[A_YI].as<double>(),
                      ctx->arr[A_ZI].as<double>()};
    TRY(dev_done(ctx, bhq::launch_unpack(&x[0][0], ni, 3, out, s), s, "set_i_dev"));
    ctx->have_i = true;
    return BHQ_OK;
}

int bhq_set_eps2_i_dev(bhq_ctx *ctx, int64_t ni, const double *eps2, void *stream)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "set_eps2_i_dev before set_groups");
    if (ni != ctx->ni)
        return ctx->fail(BHQ_E_RANGE, "set_eps2_i_dev: ni %lld != %lld", (long long)ni,
                         (long long)ctx->ni);
    if (ni > 0) {
        if (!eps2) return ctx->fail(BHQ_E_ARG, "eps2 is NULL");
        TRY(ctx->select());
        TRY(check_device_range(ctx, eps2, (size_t)ni * 8, "eps2"));
        hipStream_t s = static_cast<hipStream_t>(stream);
        ctx->quiesce();
        TRY(dev_check(ctx, s, "set_eps2_i_dev", [&](unsigned *f) {
            return bhq::launch_check_f64(eps2, ni, true, f, s);
        }));
        TRY(dev_done(ctx, hipMemcpyAsync(ctx->arr[A_E2I].p, eps2, (size_t)ni * 8,
                                         hipMemcpyDeviceToDevice, s),
                     s, "set_eps2_i_dev"));
    }
    ctx->eps_mode = 2;
    return BHQ_OK;
}

int bhq_set_jp_dev(bhq_ctx *ctx, int64_t adr, int64_t n, const double (*x)[3],
                   const double *m, void *stream)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "set_jp_dev before set_groups");
    if (adr < 0 || n < 0) return ctx->fail(BHQ_E_ARG, "negative adr or n");
    if (adr + n > ctx->njp)
        return ctx->fail(BHQ_E_RANGE, "set_jp_dev: adr + n = %lld > njp = %lld",
                         (long long)(adr + n), (long long)ctx->njp);
    if (n > 0 && (!x || !m)) return ctx->fail(BHQ_E_ARG, "x or m is NULL");
    TRY(ctx->select());
    if (n > 0) {
        TRY(check_device_range(ctx, x, (size_t)n * 24, "x"));
        TRY(check_device_range(ctx, m, (size_t)n * 8, "m"));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->quiesce();
    TRY(dev_check(ctx, s, "set_jp_dev", [&](unsigned *f) {
        hipError_t e = bhq::launch_check_f64(&x[0][0], 3 * n, false, f, s);
        if (e == hipSuccess) e = bhq::launch_check_f64(m, n, false, f, s);
        return e;
    }));
    TRY(ctx->use_materialised());
    double *out[3] = {ctx->arr[A_JPX].as<double>() + adr, ctx->arr[A_JPY].as<double>() + adr,
                      ctx->arr[A_JPZ].as<double>() + adr};
    hipError_t e = bhq::launch_unpack(&x[0][0], n, 3, out, s);
    if (e == hipSuccess && n > 0)
        e = hipMemcpyAsync(ctx->arr[A_JPM].as<double>() + adr, m, (size_t)n * 8,
                           hipMemcpyDeviceToDevice, s);
    TRY(dev_done(ctx, e, s, "set_jp_dev"));
    ctx->have_jp = true;
    return BHQ_OK;
}

int bhq_set_jc_dev(bhq_ctx *ctx, int64_t adr, int64_t n, const double (*x)[3],
                   const double *m, const double (*q)[6], const double *trace, void *stream)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "set_jc_dev before set_groups");
    if (adr < 0 || n < 0) return ctx->fail(BHQ_E_ARG, "negative adr or n");
    if (adr + n > ctx->njc)
        return ctx->fail(BHQ_E_RANGE, "set_jc_dev: adr + n = %lld > njc = %lld",
                         (long long)(adr + n), (long long)ctx->njc);
    if (n > 0 && (!x || !m || !q)) return ctx->fail(BHQ_E_ARG, "x, m or q is NULL");
    TRY(ctx->select());
    if (n > 0) {
        TRY(check_device_range(ctx, x, (size_t)n * 24, "x"));
        TRY(check_device_range(ctx, m, (size_t)n * 8, "m"));
        TRY(check_device_range(ctx, q, (size_t)n * 48, "q"));
        if (trace) TRY(check_device_range(ctx, trace, (size_t)n * 8, "trace"));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->quiesce();
    TRY(dev_check(ctx, s, "set_jc_dev", [&](unsigned *f) {
        hipError_t e = bhq::launch_check_f64(&x[0][0], 3 * n, false, f, s);
        if (e == hipSuccess) e = bhq::launch_check_f64(m, n, false, f, s);
        if (e == hipSuccess) e = bhq::launch_check_f64(&q[0][0], 6 * n, false, f, s);
        if (e == hipSuccess && trace) e = bhq::launch_check_f64(trace, n, false, f, s);
        return e;
    }));
    TRY(ctx->use_materialised());
    auto col = [&](Arr a) { return ctx->arr[a].as<double>() + adr; };
    double *xo[3] = {col(A_JCX), col(A_JCY), col(A_JCZ)};
    double *qo[6] = {col(A_Q00), col(A_Q01), col(A_Q02), col(A_Q11), col(A_Q12), col(A_Q22)};
    hipError_t e = bhq::launch_unpack(&x[0][0], n, 3, xo, s);
    if (e == hipSuccess) e = bhq::launch_unpack(&q[0][0], n, 6, qo, s);
    if (e == hipSuccess && n > 0)
        e = hipMemcpyAsync(col(A_JCM), m, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && n > 0)
        e = trace ? hipMemcpyAsync(col(A_JCT), trace, (size_t)n * 8, hipMemcpyDeviceToDevice, s)
                  : bhq::launch_fill_f64(col(A_JCT), n, 0.0, s);
    TRY(dev_done(ctx, e, s, "set_jc_dev"));
    ctx->have_jc = true;
    return BHQ_OK;
}

int bhq_set_pool_particles_dev(bhq_ctx *ctx, int64_t n, const double (*x)[3],
                               const double *m, void *stream)
{
    CHECK_CTX(ctx);
    if (n < 0 || n > 0x7fffffffLL) return ctx->fail(BHQ_E_ARG, "bad pool size");
    if (n > 0 && (!x || !m)) return ctx->fail(BHQ_E_ARG, "x or m is NULL");
    TRY(ctx->select());
    if (n > 0) {
        TRY(check_device_range(ctx, x, (size_t)n * 24, "x"));
        TRY(check_device_range(ctx, m, (size_t)n * 8, "m"));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->quiesce();
    TRY(dev_check(ctx, s, "set_pool_particles_dev", [&](unsigned *f) {
        hipError_t e = bhq::launch_check_f64(&x[0][0], 3 * n, false, f, s);
        if (e == hipSuccess) e = bhq::launch_check_f64(m, n, false, f, s);
        return e;
    }));
    hipError_t e = ctx->arr[A_POOLP].reserve((size_t)n * sizeof(bhq::PartRec));
    if (e == hipSuccess)
        e = bhq::launch_pack_particles(&x[0][0], m, n, ctx->arr[A_POOLP].as<bhq::PartRec>(), s);
    TRY(dev_done(ctx, e, s, "particle pool upload"));
    ctx->npool_p = n;
    ctx->tree_order = false;
    ctx->have_jp_idx = false;
    ++ctx->args_version;
    return BHQ_OK;
}

int bhq_set_pool_cells_dev(bhq_ctx *ctx, int64_t n, const double (*x)[3], const double *m,
                           const double (*q)[6], const double *trace, void *stream)
{
    CHECK_CTX(ctx);
    if (n < 0 || n > 0x7fffffffLL) return ctx->fail(BHQ_E_ARG, "bad pool size");
    if (n > 0 && (!x || !m || !q)) return ctx->fail(BHQ_E_ARG, "x, m or q is NULL");
    TRY(ctx->select());
    if (n > 0) {
        TRY(check_device_range(ctx, x, (size_t)n * 24, "x"));
        TRY(check_device_range(ctx, m, (size_t)n * 8, "m"));
        TRY(check_device_range(ctx, q, (size_t)n * 48, "q"));
        if (trace) TRY(check_device_range(ctx, trace, (size_t)n * 8, "trace"));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->quiesce();
    TRY(dev_check(ctx, s, "set_pool_cells_dev", [&](unsigned *f) {
        hipError_t e = bhq::launch_check_f64(&x[0][0], 3 * n, false, f, s);
        if (e == hipSuccess) e = bhq::launch_check_f64(m, n, false, f, s);
        if (e == hipSuccess) e = bhq::launch_check_f64(&q[0][0], 6 * n, false, f, s);
        if (e == hipSuccess && trace) e = bhq::launch_check_f64(trace, n, false, f, s);
        return e;
    }));
    hipError_t e = ctx->arr[A_POOLC].reserve((size_t)n * sizeof(bhq::CellRec));
    if (e == hipSuccess)
        e = bhq::launch_pack_cells(&x[0][0], m, &q[0][0], trace, n,
                                   ctx->arr[A_POOLC].as<bhq::CellRec>(), s);
    TRY(dev_done(ctx, e, s, "cell pool upload"));
    ctx->npool_c = n;
    ctx->have_jc_idx = false;
    ++ctx->args_version;
    return BHQ_OK;
}

static int set_idx_dev(bhq_ctx *ctx, Arr a, int64_t total, int64_t pool, int64_t adr,
                       int64_t n, const int32_t *idx, void *stream, const char *what)
{
    if (ctx->ng < 0) return ctx->fail(BHQ_E_STATE, "%s before set_groups", what);
    if (pool < 0) return ctx->fail(BHQ_E_STATE, "%s before its pool is set", what);
    if (adr < 0 || n < 0) return ctx->fail(BHQ_E_ARG, "negative adr or n");
    if (adr + n > total)
        return ctx->fail(BHQ_E_RANGE, "%s: adr + n = %lld > %lld", what, (long long)(adr + n),
                         (long long)total);
    if (n > 0 && !idx) return ctx->fail(BHQ_E_ARG, "idx is NULL");
    TRY(ctx->select());
    if (n > 0) TRY(check_device_range(ctx, idx, (size_t)n * 4, "idx"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->quiesce();
    TRY(dev_check(ctx, s, what, [&](unsigned *f) {
        return bhq::launch_check_idx(idx, n, pool, f, s);
    }));
    TRY(ctx->use_indexed());
    if (n == 0) return BHQ_OK;
    TRY(ctx->unslot_lists());
    return dev_done(ctx, hipMemcpyAsync(ctx->arr[a].as<int32_t>() + adr, idx, (size_t)n * 4,
                                        hipMemcpyDeviceToDevice, s),
                    s, what);
}

int bhq_set_jp_idx_dev(bhq_ctx *ctx, int64_t adr, int64_t n, const int32_t *idx, void *stream)
{
    CHECK_CTX(ctx);
    TRY(set_idx_dev(ctx, A_JPIDX, ctx->njp, ctx->npool_p, adr, n, idx, stream, "set_jp_idx_dev"));
    ctx->have_jp_idx = true;
    return BHQ_OK;
}

int bhq_set_jc_idx_dev(bhq_ctx *ctx, int64_t adr, int64_t n, const int32_t *idx, void *stream)
{
    CHECK_CTX(ctx);
    TRY(set_idx_dev(ctx, A_JCIDX, ctx->njc, ctx->npool_c, adr, n, idx, stream, "set_jc_idx_dev"));
    ctx->have_jc_idx = true;
    return BHQ_OK;
}

static int device_build(bhq_ctx *ctx, int64_t nsys, const int64_t *sys_off,
                        const double *x, const double *m, const double *eps2, double theta,
                        int ncrit, int nleaf, double box, double rcut, void *stream)
{
    const int64_t n = sys_off[nsys];
    if (n < 1 || n > 0x7fffffffLL || !x || !m || !(theta >= 0.0) || !std::isfinite(theta) ||
        ncrit < 1 || nleaf < 1 || nleaf > ncrit || !(box >= 0.0) || !std::isfinite(box) ||
        !(rcut >= 0.0) || !std::isfinite(rcut))
        return ctx->fail(BHQ_E_ARG, "build_lists_device: bad argument");
    TRY(ctx->select());
    TRY(check_device_range(ctx, x, (size_t)n * 3 * sizeof(double), "x"));
    TRY(check_device_range(ctx, m, (size_t)n * sizeof(double), "m"));
    if (eps2) TRY(check_device_range(ctx, eps2, (size_t)n * sizeof(double), "eps2"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->launched) (void)hipEventSynchronize(ctx->ev1);

    bhq::TreeParams P{x, m, eps2, n, nsys, sys_off, theta, ncrit, nleaf, box, rcut};
    // A rebuild walks once into per-group slots sized from the previous
    // device build's longest lists; the slots may take up to 4 times the
    // previous lists' memory plus 256 MiB.
    P.cap_p = ctx->walk_cap_p;
    P.cap_c = ctx->walk_cap_c;
    P.spec_levels = ctx->tree_levels;
    P.spec_cells = ctx->tree_cells;
    P.slot_bytes = ctx->ng >= 0 ? bhq::slot_memory_bound(ctx->njp, ctx->njc) : 0;
    bhq::TreeOut O;
    O.i_off = &ctx->arr[A_IOFF];
    O.jp_off = &ctx->arr[A_JPOFF];
    O.jc_off = &ctx->arr[A_JCOFF];
    O.gcx = &ctx->arr[A_GCX];
    O.gcy = &ctx->arr[A_GCY];
    O.gcz = &ctx->arr[A_GCZ];
    O.xi = &ctx->arr[A_XI];
    O.yi = &ctx->arr[A_YI];
    O.zi = &ctx->arr[A_ZI];
    O.e2i = &ctx->arr[A_E2I];
    O.pool_p = &ctx->arr[A_POOLP];
    O.pool_c = &ctx->arr[A_POOLC];
    O.jp_idx = &ctx->arr[A_JPIDX];
    O.jc_idx = &ctx->arr[A_JCIDX];
    O.order = &ctx->arr[A_TORDER];
    O.buf = ctx->tbuf;
    ctx->ng = -1;  // no valid lists unless the build completes
    ++ctx->args_version;
    std::string msg;
    const int rc = bhq::build_tree_lists(P, O, s, &msg);
    if (rc != BHQ_OK) return ctx->fail(rc, "%s", msg.c_str());

    const size_t D = sizeof(double);
    const struct { Arr a; size_t bytes; } need[] = {
        {A_E2I, (size_t)n * D}, {A_AX, (size_t)n * D}, {A_AY, (size_t)n * D},
        {A_AZ, (size_t)n * D}, {A_POT, (size_t)n * D},
    };
    for (auto &q : need) {
        // A_E2I already holds the gathered softening when eps2 was given
        if (q.a == A_E2I && eps2) continue;
        hipError_t e = ctx->arr[q.a].reserve(q.bytes);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipMalloc");
    }
    ctx->off_stale = true;
    ctx->walk_cap_p = bhq::next_slot_cap(ctx->walk_cap_p, O.max_p);
    ctx->walk_cap_c = bhq::next_slot_cap(ctx->walk_cap_c, O.max_c);
    ctx->tree_levels = O.nlevels;
    ctx->tree_cells = O.ncell;
    ctx->build_info[0] = O.one_walk ? 1 : 0;
    ctx->build_info[1] = O.max_p;
    ctx->build_info[2] = O.max_c;
    ctx->ng = O.ng;
    ctx->ni = n;
    ctx->njp = O.njp;
    ctx->njc = O.njc;
    ctx->have_i = true;
    ctx->have_jp = ctx->have_jc = ctx->have_t = false;
    ctx->list_mode = 2;
    ctx->list_slot_p = O.slot_p;
    ctx->list_slot_c = O.slot_c;
    ctx->npool_p = n;
    ctx->npool_c = O.ncell;
    ctx->have_jp_idx = ctx->have_jc_idx = true;
    ctx->tree_order = true;
    if (eps2)
        ctx->eps_mode = 2;
    else if (ctx->eps_mode == 2)
        ctx->eps_mode = 0;
    ctx->nslots = 0;
    int orc;
    if (ctx->order_mode == BHQ_ORDER_XCD &&
        bhq::plan_order_device_supported(ctx->order_window, ctx->order_tail)) {
        // the offsets are on the device already: plan there
        int64_t ns = 0;
        orc = bhq::plan_order_device(O.ng, ctx->arr[A_IOFF].as<int64_t>(),
                                     ctx->arr[A_JPOFF].as<int64_t>(),
                                     ctx->arr[A_JCOFF].as<int64_t>(), ctx->order_window,
                                     ctx->order_tail, BHQ_XCDS, ctx->arr[A_ORDER],
                                     ctx->arr[A_OSCRATCH], &ns, s, &msg);
        if (orc == BHQ_OK) {
            ctx->nslots = ns;
            ++ctx->args_version;
        } else {
            ctx->fail(orc, "%s", msg.c_str());
        }
    } else {
        orc = ctx->upload_order();
    }
    if (orc != BHQ_OK) {
        ctx->ng = -1;
        return orc;
    }
    if (ctx->eps_mode == 1) TRY(ctx->fill_eps_uniform(s));
    return BHQ_OK;
}

int bhq_build_lists_device(bhq_ctx *ctx, int64_t n, const double *x,
                           const double *m, double theta, int ncrit, int nleaf,
                           double box, double rcut, void *stream)
{
    CHECK_CTX(ctx);
    if (n < 1 || n > 0x7fffffffLL) return ctx->fail(BHQ_E_ARG, "build_lists_device: bad n");
    const int64_t off[2] = {0, n};
    return device_build(ctx, 1, off, x, m, nullptr, theta, ncrit, nleaf, box, rcut, stream);
}

int bhq_build_lists_device_batch(bhq_ctx *ctx, int64_t nsys, const int64_t *sys_off,
                                 const double *x, const double *m, const double *eps2,
                                 double theta, int ncrit, int nleaf, void *stream)
{
    CHECK_CTX(ctx);
    if (nsys < 1 || nsys > (1 << 20) || !sys_off || sys_off[0] != 0)
        return ctx->fail(BHQ_E_ARG, "build_lists_device_batch: bad systems");
    for (int64_t q = 0; q < nsys; ++q)
        if (sys_off[q + 1] <= sys_off[q])
            return ctx->fail(BHQ_E_RANGE, "build_lists_device_batch: sys_off not strictly "
                                          "increasing at %lld", (long long)q);
    if (sys_off[nsys] > 0x7fffffffLL)
        return ctx->fail(BHQ_E_ARG, "build_lists_device_batch: too many particles");
    return device_build(ctx, nsys, sys_off, x, m, eps2, theta, ncrit, nleaf, 0.0, 0.0, stream);
}

int bhq_get_lists_sizes(const bhq_ctx *ctx, int64_t out[4])
{
    if (!ctx || !out) return BHQ_E_ARG;
    if (ctx->ng < 0 || ctx->list_mode != 2) return BHQ_E_STATE;
    out[0] = ctx->ng;
    out[1] = ctx->njp;
    out[2] = ctx->njc;
    out[3] = ctx->npool_c;
    return BHQ_OK;
}

int bhq_get_lists(bhq_ctx *ctx, int64_t *i_idx, int64_t *i_off,
                  int64_t *jp_off, int64_t *jp_idx, int64_t *jc_off,
                  int32_t *jc_idx)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0 || ctx->list_mode != 2 ||
        (ctx->njp > 0 && !ctx->have_jp_idx) || (ctx->njc > 0 && !ctx->have_jc_idx))
        return ctx->fail(BHQ_E_STATE, "get_lists: no index lists set");
    if (i_idx && !ctx->tree_order)
        return ctx->fail(BHQ_E_STATE, "get_lists: the particle order is not "
                                      "known for lists set entry by entry");
    TRY(ctx->select());
    if (ctx->launched) (void)hipEventSynchronize(ctx->ev1);
    TRY(ctx->host_offsets());
    const size_t ng1 = (size_t)ctx->ng + 1;
    if (i_off) std::memcpy(i_off, ctx->i_off.data(), ng1 * 8);
    if (jp_off) std::memcpy(jp_off, ctx->jp_off.data(), ng1 * 8);
    if (jc_off) std::memcpy(jc_off, ctx->jc_off.data(), ng1 * 8);
    try {
        std::vector<int32_t> ord;
        if (ctx->tree_order && (i_idx || jp_idx)) {
            ord.resize((size_t)ctx->ni);
            hipError_t e = hipMemcpy(ord.data(), ctx->arr[A_TORDER].p,
                                     (size_t)ctx->ni * 4, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return ctx->hip_fail(e, "hipMemcpy D2H");
            if (i_idx)
                for (int64_t k = 0; k < ctx->ni; ++k) i_idx[k] = ord[(size_t)k];
        }
        if (jp_idx && ctx->njp > 0) {
            std::vector<int32_t> v((size_t)ctx->njp);
            TRY(ctx->fetch_list(A_JPIDX, A_JPOFF, ctx->list_slot_p, ctx->njp, v.data()));
            for (int64_t k = 0; k < ctx->njp; ++k)
                jp_idx[k] = ctx->tree_order ? ord[(size_t)v[(size_t)k]] : v[(size_t)k];
        }
    } catch (const std::bad_alloc &) {
        return ctx->fail(BHQ_E_NOMEM, "host staging");
    }
    if (jc_idx && ctx->njc > 0)
        TRY(ctx->fetch_list(A_JCIDX, A_JCOFF, ctx->list_slot_c, ctx->njc, jc_idx));
    return BHQ_OK;
}

int bhq_get_cells(bhq_ctx *ctx, double (*com)[3], double *mass, double (*q)[6],
                  double *trace)
{
    CHECK_CTX(ctx);
    if (ctx->npool_c < 0) return ctx->fail(BHQ_E_STATE, "get_cells: no cell pool");
    TRY(ctx->select());
    if (ctx->launched) (void)hipEventSynchronize(ctx->ev1);
    const int64_t nc = ctx->npool_c;
    std::vector<bhq::CellRec> rec;
    try {
        rec.resize((size_t)nc);
    } catch (const std::bad_alloc &) {
        return ctx->fail(BHQ_E_NOMEM, "host staging");
    }
    if (nc > 0) {
        hipError_t e = hipMemcpy(rec.data(), ctx->arr[A_POOLC].p,
                                 (size_t)nc * sizeof(bhq::CellRec), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipMemcpy D2H");
    }
    for (int64_t c = 0; c < nc; ++c) {
        const bhq::CellRec &r = rec[(size_t)c];
        if (com) {
            com[c][0] = r.x;
            com[c][1] = r.y;
            com[c][2] = r.z;
        }
        if (mass) mass[c] = r.m;
        if (q) {
            q[c][0] = r.q00;
            q[c][1] = r.q01;
            q[c][2] = r.q02;
            q[c][3] = r.q11;
            q[c][4] = r.q12;
            q[c][5] = r.q22;
        }
        if (trace) trace[c] = r.t;
    }
    return BHQ_OK;
}

int bhq_get_result_device(bhq_ctx *ctx, double *a, double *pot, void *stream)
{
    CHECK_CTX(ctx);
    if (!ctx->launched || ctx->ng < 0)
        return ctx->fail(BHQ_E_STATE, "get_result_device before compute");
    if (!a) return ctx->fail(BHQ_E_ARG, "a is NULL");
    TRY(ctx->select());
    const int64_t n = ctx->ni;
    TRY(check_device_range(ctx, a, (size_t)n * 3 * sizeof(double), "a"));
    if (pot) TRY(check_device_range(ctx, pot, (size_t)n * sizeof(double), "pot"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamWaitEvent(s, ctx->ev1, 0);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamWaitEvent");
    e = bhq::launch_scatter(ctx->tree_order ? ctx->arr[A_TORDER].as<int32_t>() : nullptr, n,
                            ctx->arr[A_AX].as<double>(), ctx->arr[A_AY].as<double>(),
                            ctx->arr[A_AZ].as<double>(), ctx->arr[A_POT].as<double>(), a,
                            pot, s);
    return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, "scatter launch");
}

int bhq_sort_to_tree_order(bhq_ctx *ctx, int64_t n, int nf, void *const *fields,
                           const int *row_bytes, void *stream)
{
    CHECK_CTX(ctx);
    if (ctx->ng < 0 || !ctx->tree_order)
        return ctx->fail(BHQ_E_STATE, "sort_to_tree_order: no lists with a tree order");
    if (n != ctx->ni || nf < 0 || nf > 16 || (nf > 0 && (!fields || !row_bytes)))
        return ctx->fail(BHQ_E_ARG, "sort_to_tree_order: bad argument");
    for (int f = 0; f < nf; ++f)
        if (!fields[f] || row_bytes[f] < 8 || row_bytes[f] > 64 || row_bytes[f] % 8 != 0)
            return ctx->fail(BHQ_E_ARG, "sort_to_tree_order: field %d", f);
    if (n == 0) return BHQ_OK;
    TRY(ctx->select());
    for (int f = 0; f < nf; ++f)
        TRY(check_device_range(ctx, fields[f], (size_t)n * (size_t)row_bytes[f], "field"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // a pending force evaluation does not read these arrays; results it is
    // still writing are scattered by the order replaced below, so wait
    hipError_t e = hipStreamWaitEvent(s, ctx->ev1, 0);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamWaitEvent");
    int maxb = 8;
    for (int f = 0; f < nf; ++f) maxb = std::max(maxb, row_bytes[f]);
    e = ctx->arr[A_SORTSCRATCH].reserve((size_t)n * (size_t)maxb);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipMalloc");
    const int32_t *order = ctx->arr[A_TORDER].as<int32_t>();
    for (int f = 0; f < nf; ++f) {
        const size_t bytes = (size_t)n * (size_t)row_bytes[f];
        e = bhq::launch_gather_rows(n, row_bytes[f] / 8, fields[f], order,
                                    ctx->arr[A_SORTSCRATCH].p, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(fields[f], ctx->arr[A_SORTSCRATCH].p, bytes,
                               hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return ctx->hip_fail(e, "gather");
    }
    // the arrays are in tree order now: tree position k is row k
    e = bhq::launch_iota(ctx->arr[A_TORDER].as<int32_t>(), n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, "tree order");
}

int bhq_kick_drift(bhq_ctx *ctx, int64_t n, double *x, double *v, const double *a,
                   double dt_kick, double dt_drift, void *stream)
{
    CHECK_CTX(ctx);
    if (!std::isfinite(dt_kick) || !std::isfinite(dt_drift))
        return ctx->fail(BHQ_E_NONFINITE, "kick_drift: time step not finite");
    if (n < 0 || !v || !a || (dt_drift != 0.0 && !x))
        return ctx->fail(BHQ_E_ARG, "kick_drift: bad argument");
    if (n == 0) return BHQ_OK;
    TRY(ctx->select());
    const size_t b = (size_t)n * 3 * sizeof(double);
    TRY(check_device_range(ctx, v, b, "v"));
    TRY(check_device_range(ctx, a, b, "a"));
    if (dt_drift != 0.0) TRY(check_device_range(ctx, x, b, "x"));
    hipError_t e = bhq::launch_kick_drift(n, x, v, a, dt_kick, dt_drift,
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, "kick_drift launch");
}

int bhq_wrap_periodic(bhq_ctx *ctx, int64_t n, double *x, double box, void *stream)
{
    CHECK_CTX(ctx);
    if (n < 0 || !x || !(box > 0.0) || !std::isfinite(box))
        return ctx->fail(BHQ_E_ARG, "wrap_periodic: bad argument");
    if (n == 0) return BHQ_OK;
    TRY(ctx->select());
    TRY(check_device_range(ctx, x, (size_t)n * 3 * sizeof(double), "x"));
    hipError_t e = bhq::launch_wrap(n, x, box, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, "wrap launch");
}

int bhq_energies(bhq_ctx *ctx, int64_t n, const double *m, const double *v,
                 const double *pot, double eps, double out[2], void *stream)
{
    CHECK_CTX(ctx);
    if (n < 1 || !m || !v || !out || !(eps >= 0.0) || !std::isfinite(eps))
        return ctx->fail(BHQ_E_ARG, "energies: bad argument");
    TRY(ctx->select());
    TRY(check_device_range(ctx, m, (size_t)n * sizeof(double), "m"));
    TRY(check_device_range(ctx, v, (size_t)n * 3 * sizeof(double), "v"));
    if (pot) TRY(check_device_range(ctx, pot, (size_t)n * sizeof(double), "pot"));
    const int nb = bhq::energy_partials();
    hipError_t e = ctx->arr[A_ENERGY].reserve((size_t)(2 * nb + 2) * sizeof(double));
    if (e != hipSuccess) return ctx->hip_fail(e, "hipMalloc");
    double *part = ctx->arr[A_ENERGY].as<double>();
    hipStream_t s = static_cast<hipStream_t>(stream);
    e = bhq::launch_energies(n, m, v, pot, eps, part, part + 2 * nb, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, part + 2 * nb, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? BHQ_OK : ctx->hip_fail(e, "energies");
}

}  // extern "C"
