// stream_bench.hip -- the bandwidth the memory system delivers to plain streaming kernels,
// the practical ceiling the solver's kernels are compared with (the 8 TB/s HBM figure is
// nominal).  For arrays of one FP32 vector at 256^3 (258^3 floats, 69 MB: the Infinity
// Cache holds a few) and at 512^3 (514^3 floats, 543 MB: it holds none) it times
//   read          sum of one array
//   copy          one read, one write
//   3r1w          three reads, one write (the access pattern of a Chebyshev step)
//   3r1w-inplace  the same with the output written over the third input
// with 16-byte vector accesses per thread and grid-stride loops over three grid sizes.
// Prints one line per case: elements, grid, kind, microseconds per launch, GB/s.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                                          \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess) {                                                                        \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);                  \
            std::exit(1);                                                                              \
        }                                                                                              \
    } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void k_read(const f4 *__restrict__ a, size_t n, float *out)
{
    f4 acc = {0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc += a[i];
    const float s = acc.x + acc.y + acc.z + acc.w;
    if (s == 12345.f) out[0] = s;   // keeps the loads; the arrays hold zeros
}

__global__ void k_copy(const f4 *__restrict__ a, f4 *__restrict__ d, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        d[i] = a[i];
}

__global__ void k_3r1w(const f4 *__restrict__ a, const f4 *__restrict__ b, const f4 *c, f4 *d, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        d[i] = a[i] + 0.5f * b[i] + 0.25f * c[i];
}

int main()
{
    const size_t sizes[2] = {(size_t)258 * 258 * 258, (size_t)514 * 514 * 514};
    const size_t maxn = sizes[1];
    float *buf[4];
    for (auto &p : buf) {
        CK(hipMalloc(&p, maxn * sizeof(float)));
        CK(hipMemset(p, 0, maxn * sizeof(float)));
    }
    float *out;
    CK(hipMalloc(&out, sizeof(float)));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const int grids[3] = {2048, 8192, 32768};
    const char *names[4] = {"read", "copy", "3r1w", "3r1w-inplace"};
    const int arrays[4] = {1, 2, 4, 4};
    for (size_t n : sizes) {
        const size_t n4 = n / 4;   // whole 16-byte groups
        for (int gsz : grids) {
            for (int kind = 0; kind < 4; ++kind) {
                f4 *A = (f4 *)buf[0], *B = (f4 *)buf[1], *Cc = (f4 *)buf[2], *D = (f4 *)buf[3];
                auto run = [&]() {
                    if (kind == 0) k_read<<<gsz, 256>>>(A, n4, out);
                    else if (kind == 1) k_copy<<<gsz, 256>>>(A, D, n4);
                    else if (kind == 2) k_3r1w<<<gsz, 256>>>(A, B, Cc, D, n4);
                    else k_3r1w<<<gsz, 256>>>(A, B, Cc, Cc, n4);
                };
                for (int w = 0; w < 3; ++w) run();
                CK(hipDeviceSynchronize());
                const int reps = 20;
                CK(hipEventRecord(e0));
                for (int r = 0; r < reps; ++r) run();
                CK(hipEventRecord(e1));
                CK(hipEventSynchronize(e1));
                float ms = 0.f;
                CK(hipEventElapsedTime(&ms, e0, e1));
                const double us = ms * 1e3 / reps;
                const double bytes = (double)n4 * 16.0 * arrays[kind];
                std::printf("n %10zu grid %6d %-13s %9.2f us %8.1f GB/s\n", n, gsz, names[kind], us, bytes / us * 1e-3);
            }
        }
    }
    for (auto p : buf) CK(hipFree(p));
    CK(hipFree(out));
    return 0;
}
