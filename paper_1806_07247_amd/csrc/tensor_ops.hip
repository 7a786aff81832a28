// Tensor operations of the toolbox that need no Fourier-domain work:
// conjugate transpose (Definition 2.2) and the identity tensor
// (Definition 2.3), on tube-major real tensors.
#include "tp_internal.h"

namespace tp {
namespace {

// A^T of a real n1 x n2 x n3 tensor: frontal slices transposed, slices 2..n3
// reversed, i.e. out(j, i, t) = A(i, j, (n3 - t) mod n3).  One thread per
// output tube; each thread reads one input tube and writes one output tube,
// both contiguous.
__global__ __launch_bounds__(256) void k_tran(const float* __restrict__ a, float* __restrict__ out, int n1, int n2,
                                              int n3)
{
    const long long ntubes = (long long)n1 * n2;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < ntubes;
         q += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(q / n1), i = (int)(q % n1);  // output tube (j, i)
        const float* src = a + ((long long)i * n2 + j) * n3;
        float* dst = out + q * n3;
        dst[0] = src[0];
        for (int t = 1; t < n3; ++t) dst[t] = src[n3 - t];
    }
}

// the n x n x n3 identity: first frontal slice I_n, the others zero
__global__ __launch_bounds__(256) void k_teye(float* __restrict__ out, int n, int n3)
{
    const long long total = (long long)n * n * n3;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long q = e / n3;
        const int t = (int)(e % n3);
        out[e] = (t == 0 && q / n == q % n) ? 1.0f : 0.0f;
    }
}

int grid_of(long long work)
{
    const long long g = (work + 255) / 256;
    return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_tran(const float* a, float* out, int n1, int n2, int n3, hipStream_t s)
{
    trace_work(0.0, 8.0 * n1 * n2 * n3);
    k_tran<<<grid_of((long long)n1 * n2), 256, 0, s>>>(a, out, n1, n2, n3);
    return hipGetLastError();
}

hipError_t launch_teye(float* out, int n, int n3, hipStream_t s)
{
    trace_work(0.0, 4.0 * n * n * n3);
    k_teye<<<grid_of((long long)n * n * n3), 256, 0, s>>>(out, n, n3);
    return hipGetLastError();
}

}  // namespace tp
