// Measurement probes: the two ceilings a forest walk is held against.
//
//  stream_copy_kernel   reads and writes a buffer once, 16 bytes per lane per
//                       step, coalesced: the HBM stream rate.
//  gather_chase_kernel  dependent random fetches: every lane follows `chains`
//                       independent pointer chains through a buffer laid out
//                       as one cycle over all its elements, loading each
//                       element whole (16, 48 or 64 bytes) and taking the
//                       next index from its first word.  The rate of such
//                       fetches against the working-set size is the ceiling
//                       of a walk whose every step needs the previous one,
//                       as a tree walk does.  With a working set that fits
//                       every CU's L1 (16 KB, say) and 8 chains per lane it
//                       is the vector-memory ceiling: the most block fetches
//                       per second the load path returns at all.
//
// The cycle: element i points to (a i + c) mod n with n a power of two, a = 1
// mod 4 and c odd, which visits all n elements once per period (Hull-Dobell),
// spreading consecutive fetches over the buffer.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fp_internal.h"

namespace {

__global__ void stream_copy_kernel(const uint4* __restrict__ a, uint4* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// element i of `words`-word elements: word 0 = next index
__global__ void gather_init_kernel(uint32_t* __restrict__ buf, uint32_t n, uint32_t words, uint32_t a, uint32_t c) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint32_t* e = buf + (size_t)i * words;
        e[0] = (a * i + c) & (n - 1u);
        for (uint32_t w = 1; w < words; w++) e[w] = i ^ w;
    }
}

// CHAINS independent chains per lane; indices are masked to [0, n) whatever
// the buffer holds, so every load stays inside it.  `sink` (word 1 of element
// 0, never read as an index) is written only if the loaded values combine to
// one particular constant, which keeps the loads from being optimised away.
template <int PIECES, int CHAINS>
__global__ __launch_bounds__(1024) void gather_chase_kernel(const uint4* __restrict__ buf, uint32_t n, int32_t steps,
                                                            uint32_t* __restrict__ sink) {
    const uint32_t mask = n - 1u, lane_id = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t idx[CHAINS], acc = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; c++) idx[c] = (lane_id * 2654435761u + (uint32_t)c * 40503u) & mask;
    for (int32_t s = 0; s < steps; s++) {
        uint4 v[CHAINS][PIECES];
#pragma unroll
        for (int c = 0; c < CHAINS; c++)
#pragma unroll
            for (int p = 0; p < PIECES; p++) v[c][p] = buf[(size_t)idx[c] * PIECES + p];
#pragma unroll
        for (int c = 0; c < CHAINS; c++) {
            idx[c] = v[c][0].x & mask;
#pragma unroll
            for (int p = 0; p < PIECES; p++) acc ^= v[c][p].y ^ v[c][p].z ^ v[c][p].w;
        }
    }
    uint32_t all = acc;
#pragma unroll
    for (int c = 0; c < CHAINS; c++) all ^= idx[c];
    if (all == 0x9e3779b9u) sink[0] = all;
}

template <int PIECES>
void launch_chase(int chains, unsigned blocks, unsigned threads, hipStream_t s, const uint4* b, uint32_t n,
                  int32_t steps, uint32_t* sink) {
    if (chains == 1) hipLaunchKernelGGL((gather_chase_kernel<PIECES, 1>), dim3(blocks), dim3(threads), 0, s, b, n, steps, sink);
    else if (chains == 2) hipLaunchKernelGGL((gather_chase_kernel<PIECES, 2>), dim3(blocks), dim3(threads), 0, s, b, n, steps, sink);
    else if (chains == 4) hipLaunchKernelGGL((gather_chase_kernel<PIECES, 4>), dim3(blocks), dim3(threads), 0, s, b, n, steps, sink);
    else hipLaunchKernelGGL((gather_chase_kernel<PIECES, 8>), dim3(blocks), dim3(threads), 0, s, b, n, steps, sink);
}

template <typename Launch>
int timed(hipStream_t s, double* ms, Launch&& launch) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fp_set_error(FP_EHIP, "hipEventCreate failed");
    }
    int rc = launch();  // warm-up
    if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = fp_set_error(FP_EHIP, "hipEventRecord failed");
    if (!rc) rc = launch();
    if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = fp_set_error(FP_EHIP, "hipEventRecord failed");
    float f = 0.0f;
    if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&f, e0, e1) != hipSuccess))
        rc = fp_set_error(FP_EHIP, "timing the probe failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = f;
    return rc;
}

int check(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FP_OK : fp_set_error(FP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" int fp_probe_stream(const void* src_dev, void* dst_dev, uint64_t bytes, double* gbps, void* stream_v) {
    fp_clear_error();
    if (!src_dev || !dst_dev || !gbps) return fp_set_error(FP_EINVAL, "NULL argument");
    if (bytes < 16 || bytes % 16 || reinterpret_cast<uintptr_t>(src_dev) % 16 || reinterpret_cast<uintptr_t>(dst_dev) % 16)
        return fp_set_error(FP_EINVAL, "bytes must be a positive multiple of 16 and both buffers 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream_v);
    const int64_t n = (int64_t)(bytes / 16);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    double ms = 0;
    int rc = timed(s, &ms, [&] {
        hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(256), 0, s, static_cast<const uint4*>(src_dev),
                           static_cast<uint4*>(dst_dev), n);
        return check("stream_copy_kernel");
    });
    if (rc) return rc;
    *gbps = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;  // read + write
    return FP_OK;
}

extern "C" int fp_probe_gather(void* buf_dev, uint64_t bytes, int32_t fetch_bytes, int32_t chains, int32_t steps,
                               double* fetches_per_s, void* stream_v) {
    fp_clear_error();
    if (!buf_dev || !fetches_per_s) return fp_set_error(FP_EINVAL, "NULL argument");
    if (fetch_bytes != 16 && fetch_bytes != 48 && fetch_bytes != 64)
        return fp_set_error(FP_EINVAL, "fetch_bytes must be 16, 48 or 64");
    if ((chains != 1 && chains != 2 && chains != 4 && chains != 8) || steps < 1)
        return fp_set_error(FP_EINVAL, "chains must be 1, 2, 4 or 8 and steps >= 1");
    if (reinterpret_cast<uintptr_t>(buf_dev) % 16) return fp_set_error(FP_EINVAL, "buffer not 16-byte aligned");
    // the largest power-of-two element count that fits, at most 2^31 elements
    uint64_t n = 1;
    while (n * 2 * (uint64_t)fetch_bytes <= bytes && n < (1ull << 31)) n *= 2;
    if (n * (uint64_t)fetch_bytes > bytes || n < 64) return fp_set_error(FP_EINVAL, "buffer holds fewer than 64 elements");
    hipStream_t s = static_cast<hipStream_t>(stream_v);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fp_set_error(FP_EHIP, "device query failed");
    const uint32_t words = (uint32_t)fetch_bytes / 4;
    hipLaunchKernelGGL(gather_init_kernel, dim3((unsigned)std::min<uint64_t>((n + 255) / 256, 65536)), dim3(256), 0, s,
                       static_cast<uint32_t*>(buf_dev), (uint32_t)n, words, 2654435761u /* = 1 mod 4 */, 12345u);
    int rc = check("gather_init_kernel");
    if (rc) return rc;
    // a full GPU of lanes: 8 waves per SIMD, 4 SIMDs per CU
    const unsigned threads = 1024, blocks = (unsigned)std::max(1, cus) * 2;
    uint32_t* sink = static_cast<uint32_t*>(buf_dev) + 1;  // word 1 of element 0: never an index
    double ms = 0;
    rc = timed(s, &ms, [&] {
        const uint4* b = static_cast<const uint4*>(buf_dev);
        if (fetch_bytes == 16) launch_chase<1>(chains, blocks, threads, s, b, (uint32_t)n, steps, sink);
        else if (fetch_bytes == 48) launch_chase<3>(chains, blocks, threads, s, b, (uint32_t)n, steps, sink);
        else launch_chase<4>(chains, blocks, threads, s, b, (uint32_t)n, steps, sink);
        return check("gather_chase_kernel");
    });
    if (rc) return rc;
    *fetches_per_s = (double)blocks * threads * chains * (double)steps / (ms * 1e-3);
    return FP_OK;
}
