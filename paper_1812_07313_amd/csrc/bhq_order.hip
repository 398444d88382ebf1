// bhq_order.hip -- the XCD dispatch order (launch slot table) computed on
// the GPU for lists that are already in device memory.  The steps and the
// arithmetic are those of the host planner (plan_order in bhq_api.cpp):
//   cost c_g = ni_g (100 njp_g + 265 njc_g + 100), in 64-bit integers;
//   B_g = sum of c_h over h < g (exact prefix sums), T = B_ng;
//   piece x_g = floor((2 B_g + c_g) / (2 T) * xcds), in FP64 with the same
//   operations, clamped to [0, xcds - 1]: contiguous pieces of equal cost;
//   in each piece, windows of `window` consecutive groups and one window of
//   its last `tail` groups, each sorted by cost, largest first (ties in
//   group order);
//   slot b of the table holds entry b / xcds of piece b % xcds, or -1.
// So the table is the host planner's, entry for entry.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "bhq.h"
#include "bhq_internal.h"

namespace bhq {

namespace {

constexpr int kBlock = 256;
constexpr int kSortMax = 1024;  // largest window sorted by one block

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_cost(int64_t ng, const int64_t *i_off,
                                                 const int64_t *jp_off, const int64_t *jc_off,
                                                 uint64_t *cost)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g > ng) return;
    cost[g] = g < ng ? order_cost(i_off[g + 1] - i_off[g], jp_off[g + 1] - jp_off[g],
                                  jc_off[g + 1] - jc_off[g])
                     : 0;  // the exclusive scan then ends with the total
}

__global__ __launch_bounds__(kBlock) void k_piece(int64_t ng, const uint64_t *cost,
                                                  const uint64_t *before, int xcds,
                                                  int32_t *piece)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= ng) return;
    piece[g] = order_piece(before[g], cost[g], before[ng], xcds, g, ng);
}

// start[p] = first group of piece p (pieces are contiguous and in order);
// start[xcds] = ng.
__global__ __launch_bounds__(kBlock) void k_starts(int64_t ng, const int32_t *piece, int xcds,
                                                   int64_t *start)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= ng) return;
    const int x = piece[g];
    const int xp = g > 0 ? piece[g - 1] : -1;
    for (int p = xp + 1; p <= x; ++p) start[p] = g;
    if (g == ng - 1)
        for (int p = x + 1; p <= xcds; ++p) start[p] = ng;
}

__global__ __launch_bounds__(kBlock) void k_fill(int32_t *v, int64_t n, int32_t val)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n) v[k] = val;
}

// One block per window: {first group, length, piece, position of the first
// group in its piece}.  Bitonic sort in LDS by (cost descending, group
// ascending), then the groups go to their slots.
struct Window {
    int32_t first, len, piece, pos;
};

__global__ __launch_bounds__(kBlock) void k_window_sort(const Window *win, const uint64_t *cost,
                                                        int xcds, int32_t *order)
{
    __shared__ uint64_t sc[kSortMax];
    __shared__ int32_t sg[kSortMax];
    const Window w = win[blockIdx.x];
    int n2 = 1;
    while (n2 < w.len) n2 <<= 1;
    for (int i = threadIdx.x; i < n2; i += kBlock) {
        // padding sorts last: cost 0 and the largest group index
        sc[i] = i < w.len ? cost[w.first + i] : 0;
        sg[i] = i < w.len ? w.first + i : 0x7fffffff;
    }
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n2; i += kBlock) {
                const int j = i ^ stride;
                if (j > i) {
                    // a before b: larger cost, then smaller group index
                    const bool up = (i & size) == 0;
                    const bool ab = sc[i] > sc[j] || (sc[i] == sc[j] && sg[i] < sg[j]);
                    if (ab != up) {
                        const uint64_t c = sc[i];
                        sc[i] = sc[j];
                        sc[j] = c;
                        const int32_t g = sg[i];
                        sg[i] = sg[j];
                        sg[j] = g;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < w.len; i += kBlock)
        order[(int64_t)(w.pos + i) * xcds + w.piece] = sg[i];
}

}  // namespace

bool plan_order_device_supported(int window, int tail)
{
    return window >= 1 && window <= kSortMax && tail >= 0 && tail <= kSortMax;
}

int plan_order_device(int64_t ng, const int64_t *i_off, const int64_t *jp_off,
                      const int64_t *jc_off, int window, int tail, int xcds, DevArray &order,
                      DevArray &scratch, int64_t *nslots, hipStream_t s, std::string *what)
{
    auto fail = [&](hipError_t e, const char *where) {
        *what = std::string(where) + ": " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? BHQ_E_NOMEM : BHQ_E_HIP;
    };
#define OSTEP(expr, where)                          \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return fail(e_, where); \
    } while (0)
    if (ng < 1 || xcds < 1 || xcds > 64 || !plan_order_device_supported(window, tail)) {
        *what = "device order: bad argument";
        return BHQ_E_ARG;
    }
    // scratch: cost[ng + 1], before[ng + 1] (uint64), piece[ng] (int32),
    // start[xcds + 1] (int64), scan temporaries
    const size_t ncost = (size_t)(ng + 1) * 8, npiece = (size_t)ng * 4;
    const size_t nstart = (size_t)(xcds + 1) * 8;
    size_t scan_bytes = 0;
    OSTEP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (uint64_t *)nullptr,
                                           (uint64_t *)nullptr, (int)(ng + 1), s),
          "order scan size");
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t o_before = up(ncost), o_piece = o_before + up(ncost);
    const size_t o_start = o_piece + up(npiece), o_scan = o_start + up(nstart);
    // windows: at most ng / window + 2 per piece
    const size_t maxwin = (size_t)(ng / window) + 2 * (size_t)xcds + 1;
    const size_t o_win = o_scan + up(scan_bytes);
    OSTEP(scratch.reserve(o_win + maxwin * sizeof(Window)), "order scratch");
    char *base = scratch.as<char>();
    uint64_t *cost = (uint64_t *)base, *before = (uint64_t *)(base + o_before);
    int32_t *piece = (int32_t *)(base + o_piece);
    int64_t *start = (int64_t *)(base + o_start);
    hipLaunchKernelGGL(k_cost, dim3(blocks(ng + 1)), dim3(kBlock), 0, s, ng, i_off, jp_off,
                       jc_off, cost);
    OSTEP(hipGetLastError(), "order cost");
    OSTEP(hipcub::DeviceScan::ExclusiveSum(base + o_scan, scan_bytes, cost, before,
                                           (int)(ng + 1), s),
          "order scan");
    hipLaunchKernelGGL(k_piece, dim3(blocks(ng)), dim3(kBlock), 0, s, ng, cost, before, xcds,
                       piece);
    OSTEP(hipGetLastError(), "order pieces");
    hipLaunchKernelGGL(k_starts, dim3(blocks(ng)), dim3(kBlock), 0, s, ng, piece, xcds, start);
    OSTEP(hipGetLastError(), "order pieces");
    std::vector<int64_t> hs((size_t)xcds + 1);
    OSTEP(hipMemcpyAsync(hs.data(), start, nstart, hipMemcpyDeviceToHost, s), "order copy");
    OSTEP(hipStreamSynchronize(s), "order sync");

    // windows of every piece, as the host planner cuts them
    std::vector<Window> win;
    int64_t longest = 0;
    for (int p = 0; p < xcds; ++p) {
        const int64_t k = hs[(size_t)p + 1] - hs[(size_t)p];
        longest = std::max(longest, k);
        const int64_t body = k > tail ? k - tail : 0;
        for (int64_t w = 0; w < body; w += window)
            win.push_back({(int32_t)(hs[(size_t)p] + w), (int32_t)(std::min(body, w + window) - w),
                           p, (int32_t)w});
        if (body < k)
            win.push_back({(int32_t)(hs[(size_t)p] + body), (int32_t)(k - body), p,
                           (int32_t)body});
    }
    const int64_t ns = longest * xcds;
    if (win.size() > maxwin) {
        *what = "device order: window table";
        return BHQ_E_RANGE;
    }
    Window *dwin = (Window *)(base + o_win);
    OSTEP(hipMemcpyAsync(dwin, win.data(), win.size() * sizeof(Window), hipMemcpyHostToDevice, s),
          "order copy");
    OSTEP(order.reserve((size_t)ns * 4), "order table");
    hipLaunchKernelGGL(k_fill, dim3(blocks(ns)), dim3(kBlock), 0, s, order.as<int32_t>(), ns, -1);
    OSTEP(hipGetLastError(), "order fill");
    hipLaunchKernelGGL(k_window_sort, dim3((unsigned)win.size()), dim3(kBlock), 0, s, dwin, cost,
                       xcds, order.as<int32_t>());
    OSTEP(hipGetLastError(), "order sort");
    // the window table is host memory read by the copy above
    OSTEP(hipStreamSynchronize(s), "order sync");
    *nslots = ns;
    return BHQ_OK;
#undef OSTEP
}

}  // namespace bhq
