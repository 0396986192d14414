// Stream-bandwidth calibration for the roofline of the HBM-bound kernels
// (not part of the method): plain and nontemporal write and read streams over
// a caller buffer, 16-byte accesses, each workgroup of BLOCK threads covering
// one contiguous 16 KB chunk, which is the per-instance tile of the K = 64
// plate kernels.  They give the rates the chip sustains for such streams,
// against which those kernels are judged next to the 8 TB/s HBM peak.
#include "qem_internal.h"
#include "dev_common.h"

namespace qemk {

namespace {

constexpr long PROBE_CHUNK_F4 = (16 << 10) / 16;   // float4s per workgroup chunk

template <bool NT>
__global__ void __launch_bounds__(BLOCK) k_probe_write(f32x4_t* __restrict__ p) {
    f32x4_t* q = p + static_cast<long>(blockIdx.x) * PROBE_CHUNK_F4;
    const f32x4_t x = {1.f, 2.f, 3.f, 4.f};
    for (long e = threadIdx.x; e < PROBE_CHUNK_F4; e += BLOCK) {
        if (NT) __builtin_nontemporal_store(x, q + e);
        else q[e] = x;
    }
}

// Every float4 of the chunk is loaded and summed; the sum is stored only if it
// is a NaN, which the buffers this runs on (filled by k_probe_write) never
// produce, so the stream is reads only.
template <bool NT>
__global__ void __launch_bounds__(BLOCK) k_probe_read(const f32x4_t* __restrict__ p, float* __restrict__ sink) {
    const f32x4_t* q = p + static_cast<long>(blockIdx.x) * PROBE_CHUNK_F4;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (long e = threadIdx.x; e < PROBE_CHUNK_F4; e += BLOCK) acc += NT ? __builtin_nontemporal_load(q + e) : q[e];
    const float s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (s != s) sink[0] = s;
}

}  // namespace

hipError_t stream_probe(hipStream_t s, void* buf, size_t bytes, int mode, float* sink) {
    const size_t chunk = static_cast<size_t>(PROBE_CHUNK_F4) * 16;
    if (!buf || bytes < chunk || bytes % chunk != 0 || bytes / chunk > 0x7fffffffu || mode < 0 || mode > 3 ||
        (mode >= 2 && !sink))
        return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(bytes / chunk));
    f32x4_t* p = static_cast<f32x4_t*>(buf);
    switch (mode) {
        case 0: hipLaunchKernelGGL(k_probe_write<false>, grid, dim3(BLOCK), 0, s, p); break;
        case 1: hipLaunchKernelGGL(k_probe_write<true>, grid, dim3(BLOCK), 0, s, p); break;
        case 2: hipLaunchKernelGGL(k_probe_read<false>, grid, dim3(BLOCK), 0, s, p, sink); break;
        default: hipLaunchKernelGGL(k_probe_read<true>, grid, dim3(BLOCK), 0, s, p, sink); break;
    }
    return hipGetLastError();
}

}  // namespace qemk
