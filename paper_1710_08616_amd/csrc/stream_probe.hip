// stream_probe.hip -- achievable HBM bandwidth on this GPU for the access
// mixes the step uses (a measurement aid, built next to the library).
//
//   copy      : read 1 array, write 1 array            (float4 per thread)
//   mix12x5   : read 12 arrays, write 5 arrays         (the short step's mix)
//   mix12x5nt : the same with non-temporal loads and stores
//
// Each kernel is timed with HIP events over `reps` launches; bandwidth is
// (bytes read + bytes written) / time.  Usage: stream_probe [mib_per_array] [reps]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                        \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));         \
            std::exit(1);                                                               \
        }                                                                               \
    } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));
#define float4 f4

struct Ptrs {
    const float4 *in[12];
    float4 *out[5];
};

__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ a, float4 *__restrict__ b,
                                              size_t n)
{
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
         q += (size_t)gridDim.x * blockDim.x)
        b[q] = a[q];
}

template <bool NT>
__global__ __launch_bounds__(256) void k_mix(Ptrs p, size_t n)
{
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
         q += (size_t)gridDim.x * blockDim.x) {
        float4 v[12];
#pragma unroll
        for (int a = 0; a < 12; ++a) {
            if constexpr (NT) {
                v[a] = __builtin_nontemporal_load(&p.in[a][q]);
            } else {
                v[a] = p.in[a][q];
            }
        }
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            const float4 r = v[o] + v[o + 5] * v[(o + 7) % 12];
            if constexpr (NT) {
                __builtin_nontemporal_store(r, &p.out[o][q]);
            } else {
                p.out[o][q] = r;
            }
        }
    }
}

int main(int argc, char **argv)
{
    const size_t mib = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 256;
    const int reps = argc > 2 ? std::atoi(argv[2]) : 10;
    const size_t bytes = mib << 20, n4 = bytes / sizeof(float4);
    std::vector<void *> bufs(17);
    for (auto &b : bufs) {
        CHECK(hipMalloc(&b, bytes));
        CHECK(hipMemset(b, 0, bytes));
    }
    Ptrs p;
    for (int a = 0; a < 12; ++a) p.in[a] = (const float4 *)bufs[a];
    for (int o = 0; o < 5; ++o) p.out[o] = (float4 *)bufs[12 + o];
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    int dev = 0, cus = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int grids[] = {cus * 8, cus * 32, (int)((n4 + 255) / 256)};
    for (int g : grids) {
        for (int kind = 0; kind < 3; ++kind) {
            auto launch = [&] {
                if (kind == 0) hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, 0, p.in[0], p.out[0], n4);
                else if (kind == 1) hipLaunchKernelGGL(k_mix<false>, dim3(g), dim3(256), 0, 0, p, n4);
                else hipLaunchKernelGGL(k_mix<true>, dim3(g), dim3(256), 0, 0, p, n4);
            };
            launch();
            CHECK(hipDeviceSynchronize());
            CHECK(hipEventRecord(e0, 0));
            for (int r = 0; r < reps; ++r) launch();
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            const double per = ms / reps;
            const double moved = (kind == 0 ? 2.0 : 17.0) * (double)bytes;
            std::printf("%-10s grid %8d  %8.3f ms  %7.0f GB/s\n",
                        kind == 0 ? "copy" : (kind == 1 ? "mix12x5" : "mix12x5nt"), g, per,
                        moved / (per * 1e-3) / 1e9);
        }
    }
    for (auto b : bufs) CHECK(hipFree(b));
    return 0;
}
