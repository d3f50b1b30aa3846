// Access-pattern ceilings for the local phases of the 2^24 transform
// (4096 x 4096 complex64, 128 MiB per buffer): how fast the memory system
// moves the bytes of a column-tile pass when the pass does no arithmetic.
//
// A local phase reads an n x W column tile of a row-major matrix (W complex
// items per row: a run of 8 W bytes, rows 32 KiB apart) and writes it back.
// This tool times exactly that load and store, with the library's
// XCD-aware tile order, for W = 4, 8 and 16 (32-, 64- and 128-byte runs),
// next to a plain contiguous copy.  "cold" cycles four buffer pairs (1 GiB)
// so that no launch finds its input in the 256 MiB MALL; "warm" reuses one
// pair, whose 256 MiB the MALL mostly holds.  A column-FFT tile can do no
// better than the no-arithmetic pass of its own pattern.
//
// Built beside this file by the package's build step (hipcc for gfx950, as
// the library); run ./access_pattern on one MI355X: one line per pattern and mode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));           \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)

namespace {

constexpr int kRows = 4096, kCols = 4096;  // complex64 items
constexpr int kThreads = 512;

// The library's tile order: the hardware deals consecutive workgroups to the
// 8 XCDs in turn; workgroups that one XCD receives own neighbouring tiles.
__device__ __forceinline__ int xcd_order(int i, int G) { return (G & 7) ? i : (i & 7) * (G >> 3) + (i >> 3); }

// One workgroup per kRows x W tile; each lane moves 16 bytes (2 items) per
// row it handles.  Every load is issued before the first store, as in a
// column-FFT tile.
template <int W, bool XCD>
__global__ __launch_bounds__(kThreads) void column_tile_pass(const float4 *__restrict__ src, float4 *__restrict__ dst)
{
    constexpr int lanes_per_row = W / 2;
    constexpr int rows_per_round = kThreads / lanes_per_row;
    constexpr int rounds = kRows / rows_per_round;
    const int tile = XCD ? xcd_order(blockIdx.x, gridDim.x) : int(blockIdx.x);
    const int r0 = threadIdx.x / lanes_per_row, c = threadIdx.x % lanes_per_row;
    float4 v[rounds];
#pragma unroll
    for (int k = 0; k < rounds; ++k)
        v[k] = src[(size_t(r0 + k * rows_per_round) * kCols + size_t(tile) * W) / 2 + c];
#pragma unroll
    for (int k = 0; k < rounds; ++k)
        dst[(size_t(tile) * kRows + size_t(r0 + k * rows_per_round)) * W / 2 + c] = v[k];
}

__global__ __launch_bounds__(kThreads) void contiguous_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                            size_t n4)
{
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n4; i += size_t(gridDim.x) * kThreads)
        dst[i] = src[i];
}

// Median of 30 single-launch times (HIP events on the null stream).
template <typename Launch>
float median_ms(Launch launch)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    launch();
    launch();
    CHECK(hipDeviceSynchronize());
    std::vector<float> ms;
    for (int r = 0; r < 30; ++r) {
        CHECK(hipEventRecord(a, nullptr));
        launch();
        CHECK(hipEventRecord(b, nullptr));
        CHECK(hipEventSynchronize(b));
        float t = 0.f;
        CHECK(hipEventElapsedTime(&t, a, b));
        ms.push_back(t);
    }
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

}  // namespace

int main()
{
    const size_t n = size_t(kRows) * kCols;
    constexpr int kPairs = 4;
    float4 *src[kPairs], *dst[kPairs];
    for (int i = 0; i < kPairs; ++i) {
        CHECK(hipMalloc(&src[i], n * 8));
        CHECK(hipMalloc(&dst[i], n * 8));
        CHECK(hipMemset(src[i], 0, n * 8));
        CHECK(hipMemset(dst[i], 0, n * 8));
    }
    const double bytes = 2.0 * double(n) * 8.0;  // read once, written once
    std::printf("pattern (4096 x 4096 complex64, %.0f MB moved per launch) | mode | us | TB/s\n", bytes / 1e6);
    for (int cold = 1; cold >= 0; --cold) {
        int next = 0;
        auto pick = [&] { return cold ? (next++ % kPairs) : 0; };
        auto report = [&](const char *name, float ms) {
            std::printf("%-44s | %s | %7.1f | %5.2f\n", name, cold ? "cold" : "warm", ms * 1e3, bytes / (ms * 1e-3) / 1e12);
            std::fflush(stdout);
        };
        report("contiguous copy", median_ms([&] {
                   const int i = pick();
                   contiguous_copy<<<4096, kThreads>>>(src[i], dst[i], n / 2);
               }));
        report("4-column tiles, 32 B runs, launch order", median_ms([&] {
                   const int i = pick();
                   column_tile_pass<4, false><<<kCols / 4, kThreads>>>(src[i], dst[i]);
               }));
        report("4-column tiles, 32 B runs, XCD order", median_ms([&] {
                   const int i = pick();
                   column_tile_pass<4, true><<<kCols / 4, kThreads>>>(src[i], dst[i]);
               }));
        report("8-column tiles, 64 B runs, XCD order", median_ms([&] {
                   const int i = pick();
                   column_tile_pass<8, true><<<kCols / 8, kThreads>>>(src[i], dst[i]);
               }));
        report("16-column tiles, 128 B runs, XCD order", median_ms([&] {
                   const int i = pick();
                   column_tile_pass<16, true><<<kCols / 16, kThreads>>>(src[i], dst[i]);
               }));
    }
    CHECK(hipDeviceSynchronize());
    for (int i = 0; i < kPairs; ++i) {
        CHECK(hipFree(src[i]));
        CHECK(hipFree(dst[i]));
    }
    return 0;
}
