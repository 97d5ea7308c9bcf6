// LDS read bandwidth of the device, measured rather than quoted: the ceiling
// that the likelihood kernel's Q staging (16-byte LDS reads of 128-byte
// blocks) is compared against.
//
// Every block holds 16 KB of LDS, 8 blocks per CU (128 KB of the 160 KB);
// each wavefront streams 16-byte reads (ds_read_b128) over its own 4 KB,
// consecutive lanes on consecutive 16-byte words (no bank conflicts), and
// folds them into four FP32 sums so that the reads stay live.  A compiler
// memory barrier in the loop makes every iteration read LDS again.
//
//     lds_peak [iterations]
//
// prints one line: bytes read per second over the device, the CU count, and
// bytes per CU per cycle at the device's reported engine clock.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int THREADS = 256;      // 4 wavefronts
constexpr int WORDS = 1024;       // 16-byte words per block: 16 KB
constexpr int BLOCKS_PER_CU = 8;  // 128 KB of LDS per CU
constexpr int UNROLL = 4;         // reads per lane per iteration

__global__ void __launch_bounds__(THREADS) k_lds_read(float* out, int iters) {
  __shared__ float4 buf[WORDS];
  for (int j = threadIdx.x; j < WORDS; j += THREADS) buf[j] = make_float4((float)j, 1.0f, 2.0f, 3.0f);
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const float4* base = buf + w * (WORDS / 4);  // this wavefront's 256 words
  float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
  for (int i = 0; i < iters; ++i) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const float4 v = base[u * 64 + l];
      if (u & 1) {
        b.x += v.x; b.y += v.y; b.z += v.z; b.w += v.w;
      } else {
        a.x += v.x; a.y += v.y; a.z += v.z; a.w += v.w;
      }
    }
  }
  const float s = a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w;
  if (s == -1.0f) out[threadIdx.x] = s;  // never true; keeps the sums (and reads) live
}

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));        \
      return 1;                                                           \
    }                                                                     \
  } while (0)

}  // namespace

int main(int argc, char** argv) {
  const int iters = argc > 1 ? std::atoi(argv[1]) : 20000;
  if (iters < 1 || iters > 10000000) {
    std::fprintf(stderr, "iterations must be in [1, 1e7]\n");
    return 2;
  }
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int n_cu = prop.multiProcessorCount;
  const int blocks = n_cu * BLOCKS_PER_CU;
  float* out = nullptr;
  CHECK(hipMalloc(&out, sizeof(float) * THREADS));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(THREADS), 0, 0, out, iters);  // warm-up
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  float best = 1e30f;
  for (int r = 0; r < 5; ++r) {
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(THREADS), 0, 0, out, iters);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) best = ms;
  }
  const double bytes = (double)blocks * THREADS * UNROLL * 16.0 * iters;
  const double bps = bytes / (best * 1e-3);
  const double mhz = prop.clockRate / 1000.0;
  std::printf("lds_read_bytes_per_s %.4g cus %d bytes_per_cu_per_cycle %.1f at %.0f MHz (best of 5, %.3f ms)\n",
              bps, n_cu, bps / n_cu / (mhz * 1e6), mhz, best);
  CHECK(hipFree(out));
  return 0;
}
