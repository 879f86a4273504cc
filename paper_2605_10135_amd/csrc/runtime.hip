// runtime.hip -- status strings, per-thread error text, device exclusive scan.
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

namespace sg {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// exclusive scan of int64 (three passes: tile sums, scan of the sums, tile
// scans plus carried prefix); deterministic.
// ---------------------------------------------------------------------------
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    // inclusive wave scan
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int i = 0; i < SCAN_THREADS / 64; ++i) {
            int64_t s = sh[i];
            sh[i] = run;
            run += s;
        }
        sh[SCAN_THREADS / 64] = run;
    }
    __syncthreads();
    int64_t r = x - v + sh[w];
    *total = sh[SCAN_THREADS / 64];
    __syncthreads();
    return r;
}

__global__ void scan_tile_sums(const int64_t* __restrict__ in, int64_t n, int64_t* __restrict__ sums) {
    __shared__ int64_t sh[SCAN_THREADS / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        if (k < n) acc += in[k];
    }
    int64_t total;
    block_exclusive_scan(acc, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void scan_tiles(const int64_t* __restrict__ in, int64_t n, const int64_t* __restrict__ carry,
                           int64_t* __restrict__ out) {
    __shared__ int64_t sh[SCAN_THREADS / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t vals[SCAN_ITEMS];
    int64_t acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        vals[i] = (k < n) ? in[k] : 0;
        acc += vals[i];
    }
    int64_t total;
    int64_t pre = block_exclusive_scan(acc, sh, &total) + (carry ? carry[blockIdx.x] : 0);
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        if (k < n) out[k] = pre;
        pre += vals[i];
    }
    // the element past the end holds the grand total
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) out[n] = pre;
}

size_t exclusive_scan_tmp_bytes(int64_t n) {
    size_t bytes = 0;
    int64_t m = n;
    while (m > SCAN_TILE) {
        int64_t tiles = (m + SCAN_TILE - 1) / SCAN_TILE;
        bytes += align_up((size_t)(tiles + 1) * 2 * sizeof(int64_t), 256);
        m = tiles;
    }
    return bytes + 256;
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s) {
    if (n <= 0) {
        fill<int64_t>(out, 0, 1, s);
        return;
    }
    int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles == 1) {
        scan_tiles<<<1, SCAN_THREADS, 0, s>>>(in, n, nullptr, out);
        SG_LAUNCH_CHECK();
        return;
    }
    int64_t* sums = static_cast<int64_t*>(tmp);
    int64_t* carry = sums + (tiles + 1);
    char* rest = static_cast<char*>(tmp) + align_up((size_t)(tiles + 1) * 2 * sizeof(int64_t), 256);
    scan_tile_sums<<<(unsigned)tiles, SCAN_THREADS, 0, s>>>(in, n, sums);
    SG_LAUNCH_CHECK();
    exclusive_scan_i64(sums, carry, tiles, rest, s);
    scan_tiles<<<(unsigned)tiles, SCAN_THREADS, 0, s>>>(in, n, carry, out);
    SG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// distance-kernel profiling (event pairs around each launch)
// ---------------------------------------------------------------------------
namespace {
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;
}  // namespace

bool profiling_on() {
    std::lock_guard<std::mutex> g(g_prof_mu);
    return g_prof_on;
}

void profile_record(hipStream_t s, bool before) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on) return;
    if (before) {
        hipEvent_t a, b;
        SG_HIP(hipEventCreate(&a));
        SG_HIP(hipEventCreate(&b));
        g_prof_events.emplace_back(a, b);
        SG_HIP(hipEventRecord(a, s));
    } else if (!g_prof_events.empty()) {
        SG_HIP(hipEventRecord(g_prof_events.back().second, s));
    }
}

}  // namespace sg

extern "C" {

sg_status sg_profile_begin(void) {
    return sg::guarded([&] {
        std::lock_guard<std::mutex> g(sg::g_prof_mu);
        for (auto& e : sg::g_prof_events) {
            hipEventDestroy(e.first);
            hipEventDestroy(e.second);
        }
        sg::g_prof_events.clear();
        sg::g_prof_on = true;
    });
}

sg_status sg_profile_end(double* kernel_ms, int64_t* launches) {
    return sg::guarded([&] {
        SG_REQUIRE(kernel_ms != nullptr && launches != nullptr, "NULL pointer");
        std::lock_guard<std::mutex> g(sg::g_prof_mu);
        double total = 0.0;
        for (auto& e : sg::g_prof_events) {
            SG_HIP(hipEventSynchronize(e.second));
            float ms = 0.f;
            SG_HIP(hipEventElapsedTime(&ms, e.first, e.second));
            total += ms;
            hipEventDestroy(e.first);
            hipEventDestroy(e.second);
        }
        *kernel_ms = total;
        *launches = (int64_t)sg::g_prof_events.size();
        sg::g_prof_events.clear();
        sg::g_prof_on = false;
    });
}

const char* sg_status_str(sg_status s) {
    switch (s) {
        case SG_OK: return "SG_OK";
        case SG_ERR_ARG: return "SG_ERR_ARG: invalid argument";
        case SG_ERR_HIP: return "SG_ERR_HIP: HIP runtime or launch failure";
        case SG_ERR_WORKSPACE: return "SG_ERR_WORKSPACE: workspace missing or too small";
        case SG_ERR_UNSUPPORTED: return "SG_ERR_UNSUPPORTED: unsupported combination";
        case SG_ERR_INTERNAL: return "SG_ERR_INTERNAL: internal failure";
        default: return "unknown sg_status";
    }
}

const char* sg_last_error(void) { return sg::get_error(); }

const char* sg_version(void) { return "sg 0.1 (gfx950)"; }

}  // extern "C"
