// LDS accumulation microbenchmark for gfx950: the throughput of the LDS
// operations a spread kernel can accumulate with, in lane-operations per
// clock per compute unit, for two address patterns:
//   random   - every lane of a wave hits an arbitrary word of the array;
//   classes  - consecutive lanes hit distinct bank classes (the layout the
//              spread's particle dealing produces): 16 classes of 64-bit
//              words or 32 of 32-bit words per 128-byte row.
// Operations: 64-bit integer add (ds_add_u64), 32-bit integer add
// (ds_add_u32), 32-bit float add (ds_add_f32) and, as the reference, plain
// 32-bit reads (ds_read_b32). Each thread holds 16 precomputed addresses and
// walks them with a per-round offset that is a multiple of 32 words (bank
// classes kept), so the loop costs two VALU operations per LDS operation.
// Blocks of 512 threads; the array is 64 KB (2 blocks per compute unit, the
// occupancy of the spread's 74 KB tile) or 32 KB (4 blocks). Prints one JSON
// line per (operation, pattern, array size). Not part of the library.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kThreads = 512;

__device__ __forceinline__ unsigned hash32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// first-round word index of address j of this lane (stride: words per element)
template <int WORDS>
__device__ __forceinline__ unsigned first_addr(int pattern, int j, int stride) {
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (pattern == 0) return (hash32(j * 4099u + threadIdx.x * 131u + blockIdx.x) % (WORDS / stride)) * stride;
    const unsigned classes = 32 / stride;
    const unsigned row = hash32(j * 977u + (lane / classes) * 31u + wave * 7u + blockIdx.x) % (WORDS / 32);
    return row * 32 + (lane % classes) * stride;
}

template <int OP, int WORDS>
__global__ void __launch_bounds__(kThreads) k_lds(int pattern, int rounds, unsigned* out) {
    __shared__ __align__(16) unsigned lds[WORDS];
    for (int i = threadIdx.x; i < WORDS; i += kThreads) lds[i] = 0;
    const int stride = OP == 0 ? 2 : 1;
    unsigned a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = first_addr<WORDS>(pattern, j, stride);
    __syncthreads();
    unsigned acc = 0;
    for (int r = 0; r < rounds; ++r) {
        const unsigned off = ((unsigned)r * 32u * 37u) & (WORDS - 1);  // a multiple of 32 words
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const unsigned w = (a[j] + off) & (WORDS - 1);
            if constexpr (OP == 0)
                atomicAdd(reinterpret_cast<unsigned long long*>(lds + w), 1ull);
            else if constexpr (OP == 1)
                atomicAdd(lds + w, 1u);
            else if constexpr (OP == 2)
                atomicAdd(reinterpret_cast<float*>(lds) + w, 1.0f);
            else
                acc += lds[w];
        }
    }
    __syncthreads();
    unsigned s = acc;
    for (int i = threadIdx.x; i < WORDS; i += kThreads) s += lds[i];
    if (s == 0x12345678u) out[blockIdx.x] = s;  // keeps the work observable
}

const char* kOps[] = {"ds_add_u64", "ds_add_u32", "ds_add_f32", "ds_read_b32"};
const char* kPatterns[] = {"random", "classes"};

template <int OP, int WORDS>
float run(int pattern, int rounds, int blocks, unsigned* out) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    k_lds<OP, WORDS><<<blocks, kThreads>>>(pattern, rounds, out);  // warm-up
    (void)hipEventRecord(e0);
    k_lds<OP, WORDS><<<blocks, kThreads>>>(pattern, rounds, out);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

template <int WORDS>
float run_op(int op, int pattern, int rounds, int blocks, unsigned* out) {
    switch (op) {
        case 0: return run<0, WORDS>(pattern, rounds, blocks, out);
        case 1: return run<1, WORDS>(pattern, rounds, blocks, out);
        case 2: return run<2, WORDS>(pattern, rounds, blocks, out);
        default: return run<3, WORDS>(pattern, rounds, blocks, out);
    }
}

}  // namespace

int main(int argc, char** argv) {
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) return 1;
    const int cus = prop.multiProcessorCount;
    const double clk_hz = prop.clockRate * 1e3;
    const int blocks = cus * 8;
    unsigned* out = nullptr;
    if (hipMalloc(&out, sizeof(unsigned) * blocks) != hipSuccess) return 1;
    for (int kb : {64, 32}) {
        for (int op = 0; op < 4; ++op) {
            for (int pat = 0; pat < 2; ++pat) {
                // the float atomics are ~15x slower: fewer rounds
                const int r = op == 2 ? rounds / 8 : rounds;
                const float ms = kb == 64 ? run_op<16384>(op, pat, r, blocks, out)
                                          : run_op<8192>(op, pat, r, blocks, out);
                const double lane_ops = (double)blocks * kThreads * r * 16;
                const double per_clk_cu = lane_ops / (ms * 1e-3) / clk_hz / cus;
                std::printf("{\"op\": \"%s\", \"pattern\": \"%s\", \"array_kb\": %d, \"ms\": %.4f, "
                            "\"lane_ops\": %.0f, \"lane_ops_per_clk_per_cu\": %.3f, \"clock_mhz\": %.0f, "
                            "\"cus\": %d}\n",
                            kOps[op], kPatterns[pat], kb, ms, lane_ops, per_clk_cu, clk_hz / 1e6, cus);
                std::fflush(stdout);
            }
        }
    }
    (void)hipFree(out);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}
