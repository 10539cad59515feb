// Allocation-free Stiefel tangent projection for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// G = D - W (W^T D + D^T W) / 2 (Sec. 2.2, eq. stiefel_gradient, real case), factor by factor, as
// stiefel_project computes it, with the one intermediate, S = W^T D (p x p, FP64), kept in a file-scope device
// array instead of the context's workspace. The array is fixed in size (kScratchDoubles doubles, 8 MiB, so
// p <= 1024) and exists once per GPU for the life of the process; its address on each device is looked up once,
// with that device current, when the first context on the device is created. Every call on a GPU reuses that GPU's
// array: S is written in full before it is read, so nothing has to be cleared between calls, but two calls that
// overlap on one GPU (different streams or contexts) race on it.
#include <array>
#include <mutex>

#include "common.h"

namespace mera {

namespace {

constexpr int64_t kScratchDoubles = (int64_t)1 << 20;  // 8 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::array<double*, kMaxDevices> g_scratch_ptr{};

constexpr int kTile = 32;

// S[i, j] = sum_r W[r, i] D[r, j] over the n rows; W, D row-major n x p. One 32 x 32 block of S per workgroup of
// 256 threads (2 x 2 outputs each), rows staged through LDS 32 at a time.
__global__ void __launch_bounds__(256) wtd_kernel(const double* __restrict__ W, const double* __restrict__ D, int n,
                                                   int p, double* __restrict__ S) {
  __shared__ double Ws[kTile][kTile + 1];
  __shared__ double Ds[kTile][kTile + 1];
  const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int r0 = 0; r0 < n; r0 += kTile) {
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
      const int r = e / kTile, c = e % kTile, row = r0 + r;
      Ws[r][c] = (row < n && i0 + c < p) ? W[(int64_t)row * p + i0 + c] : 0.0;
      Ds[r][c] = (row < n && j0 + c < p) ? D[(int64_t)row * p + j0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kTile; ++k) {
      const double w0 = Ws[k][2 * ty], w1 = Ws[k][2 * ty + 1];
      const double d0 = Ds[k][2 * tx], d1 = Ds[k][2 * tx + 1];
      acc[0][0] = fma(w0, d0, acc[0][0]);
      acc[0][1] = fma(w0, d1, acc[0][1]);
      acc[1][0] = fma(w1, d0, acc[1][0]);
      acc[1][1] = fma(w1, d1, acc[1][1]);
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int i = i0 + 2 * ty + a, j = j0 + 2 * tx + b;
      if (i < p && j < p) S[(int64_t)i * p + j] = acc[a][b];
    }
}

// G[r, j] = D[r, j] - sum_i W[r, i] (S[i, j] + S[j, i]) / 2. One 32 x 32 block of G per workgroup; each thread
// reads D only at the elements it writes, so G may alias D.
__global__ void __launch_bounds__(256) project_kernel(const double* __restrict__ W, const double* D,
                                                       const double* __restrict__ S, int n, int p, double* G) {
  __shared__ double Wt[kTile][kTile + 1];
  __shared__ double Ss[kTile][kTile + 1];
  const int r0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int i0 = 0; i0 < p; i0 += kTile) {
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
      const int r = e / kTile, c = e % kTile;
      const int row = r0 + r, i = i0 + c;
      Wt[r][c] = (row < n && i < p) ? W[(int64_t)row * p + i] : 0.0;
      // Ss[k][c]: symmetric part of S at (i0 + k, j0 + c)
      const int k = e / kTile, jj = j0 + c, ii = i0 + k;
      Ss[k][c] = (ii < p && jj < p) ? 0.5 * (S[(int64_t)ii * p + jj] + S[(int64_t)jj * p + ii]) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kTile; ++k) {
      const double w0 = Wt[2 * ty][k], w1 = Wt[2 * ty + 1][k];
      const double s0 = Ss[k][2 * tx], s1 = Ss[k][2 * tx + 1];
      acc[0][0] = fma(w0, s0, acc[0][0]);
      acc[0][1] = fma(w0, s1, acc[0][1]);
      acc[1][0] = fma(w1, s0, acc[1][0]);
      acc[1][1] = fma(w1, s1, acc[1][1]);
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int r = r0 + 2 * ty + a, j = j0 + 2 * tx + b;
      if (r < n && j < p) {
        const int64_t o = (int64_t)r * p + j;
        G[o] = D[o] - acc[a][b];
      }
    }
}

}  // namespace

int64_t noalloc_scratch_doubles() { return kScratchDoubles; }

// Looks up this device's copy of the scratch array (the device must be current). Called once per device from the
// context's creation; later calls return the stored address.
double* noalloc_scratch(int device) {
  MERA_CHECK(device >= 0 && device < kMaxDevices, MERA_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    MERA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MERA_CHECK(p != nullptr, MERA_EHIP, "no device address for the scratch array");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  return g_scratch_ptr[device];
}

// Launches the projection of every factor on `stream` (no synchronisation, no allocation). Shapes are checked by
// the caller; p * p must not exceed the scratch size.
void stiefel_project_noalloc_run(double* S, hipStream_t stream, int count, const int* n, const int* p,
                                 const double* const* W, const double* const* D, double* const* G) {
  for (int f = 0; f < count; ++f) {
    const int nf = n[f], pf = p[f];
    const int tp = (pf + kTile - 1) / kTile, tn = (nf + kTile - 1) / kTile;
    hipLaunchKernelGGL(wtd_kernel, dim3(tp, tp), dim3(256), 0, stream, W[f], D[f], nf, pf, S);
    MERA_HIP(hipGetLastError());
    hipLaunchKernelGGL(project_kernel, dim3(tp, tn), dim3(256), 0, stream, W[f], D[f], S, nf, pf, G[f]);
    MERA_HIP(hipGetLastError());
  }
}

}  // namespace mera
