// Memory-bound kernels: reductions accumulate in FP64 with a wavefront shuffle tree, then per-block partials
// are summed on the host in a fixed order (deterministic).
#include "vec.h"

#include <cmath>
#include <unordered_map>

namespace mera {

namespace {

constexpr int RED_BLOCKS = 1024;
constexpr int TPB = 256;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ inline void block_sum_store(double v, double* out) {
  __shared__ double part[TPB / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < TPB / 64; ++i) s += part[i];
    out[blockIdx.x] = s;
  }
}

template <typename TX, typename TY>
__global__ void dot_kernel(const TX* __restrict__ x, const TY* __restrict__ y, int64_t n, double* out) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)x[i] * (double)y[i];
  block_sum_store(s, out);
}

template <typename TX, typename TY>
__global__ void axpby_kernel(double a, const TX* __restrict__ x, double b, TY* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * (double)x[i];
    if (b != 0.0) v += b * (double)y[i];
    y[i] = (TY)v;
  }
}

// Several vectors of one precision per launch, passed by value with their coefficients.
constexpr int kMulti = 17;
template <typename T>
struct VecList {
  const T* v[kMulti];
  double c[kMulti];
};

// Block partials of the k dot products <w, v_j>: one pass over w, each element of w read once.
// out[j * gridDim.x + blockIdx.x] = this block's share of sum_i w[i] v_j[i].
template <typename T>
__global__ void multi_dot_kernel(VecList<T> L, int k, const T* __restrict__ w, int64_t n, double* __restrict__ out) {
  double s[kMulti];
#pragma unroll
  for (int j = 0; j < kMulti; ++j) s[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = (double)w[i];
#pragma unroll
    for (int j = 0; j < kMulti; ++j)
      if (j < k) s[j] += wi * (double)L.v[j][i];
  }
  __shared__ double part[kMulti][TPB / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kMulti; ++j)
    if (j < k) {
      const double t = wave_sum(s[j]);
      if (lane == 0) part[j][wave] = t;
    }
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double t = 0.0;
    for (int q = 0; q < TPB / 64; ++q) t += part[threadIdx.x][q];
    out[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// sums[j] = sum of the `blocks` partials of vector j, in a fixed order (one wave per vector).
__global__ void sum_partials_kernel(const double* __restrict__ part, int blocks, double* __restrict__ sums) {
  const int j = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < blocks; b += 64) t += part[(int64_t)j * blocks + b];
  t = wave_sum(t);
  if (threadIdx.x == 0) sums[j] = t;
}

// y <- b y + sum_j c_j v_j, accumulated in FP64 and rounded once (b == 0: y is not read).
template <typename T>
__global__ void multi_axpby_kernel(VecList<T> L, int k, double b, T* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double t = (b != 0.0) ? b * (double)y[i] : 0.0;
#pragma unroll
    for (int j = 0; j < kMulti; ++j)
      if (j < k) t += L.c[j] * (double)L.v[j][i];
    y[i] = (T)t;
  }
}

// y <- b y + sum_j (s c[j]) v_j with the coefficients read from device memory.
template <typename T>
__global__ void multi_axpby_dev_kernel(VecList<T> L, int k, const double* __restrict__ c, double s, double b,
                                       T* __restrict__ y, int64_t n) {
  double cj[kMulti];
#pragma unroll
  for (int j = 0; j < kMulti; ++j) cj[j] = (j < k) ? s * c[j] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double t = (b != 0.0) ? b * (double)y[i] : 0.0;
#pragma unroll
    for (int j = 0; j < kMulti; ++j)
      if (j < k) t += cj[j] * (double)L.v[j][i];
    y[i] = (T)t;
  }
}

// y = (s a) x + b y with a read from device memory.
template <typename TX, typename TY>
__global__ void axpby_dev_kernel(const double* __restrict__ a, double s, const TX* __restrict__ x, double b,
                                 TY* __restrict__ y, int64_t n) {
  const double av = s * a[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = av * (double)x[i];
    if (b != 0.0) v += b * (double)y[i];
    y[i] = (TY)v;
  }
}

template <typename T>
__global__ void add_diag_dev_kernel(T* x, int64_t dim, const double* __restrict__ c, double s) {
  const double cv = s * c[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += (int64_t)gridDim.x * blockDim.x)
    x[i * dim + i] = (T)((double)x[i * dim + i] + cv);
}

// nrm[0] = sqrt(sum of the squares in sq[0]); x <- x / nrm[0] when positive (one thread writes nrm)
template <typename T>
__global__ void normalize_dev_kernel(T* x, int64_t n, const double* __restrict__ sq, double* __restrict__ nrm) {
  const double hn = sqrt(sq[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) nrm[0] = hn;
  if (!(hn > 0.0)) return;
  const double a = 1.0 / hn;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)(a * (double)x[i]);
}

template <typename T>
VecList<T> vec_list(const VPtr* v, const double* c, int k) {
  VecList<T> L{};
  for (int j = 0; j < k; ++j) {
    L.v[j] = static_cast<const T*>(v[j].p);
    L.c[j] = c ? c[j] : 0.0;
  }
  return L;
}

// *out = the partial sums added one after another in order (as the host adds them after a copy).
__global__ void sum_partials_seq_kernel(const double* __restrict__ part, int blocks, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (int b = 0; b < blocks; ++b) t += part[b];
  out[0] = t;
}

// x <- (num / den) x, the ratio of two device scalars (the same operations as scal with the ratio formed on the host).
template <typename T>
__global__ void scal_ratio_kernel(const double* __restrict__ num, const double* __restrict__ den, T* x, int64_t n) {
  const double a = num[0] / den[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)(a * (double)x[i]);
}

// r p - r q with both products rounded before the subtraction, as the host forms it
__device__ inline double rounded_diff(double r, double p, double q) {
#pragma clang fp contract(off)
  const double rp = r * p;
  const double rq = r * q;
  return rp - rq;
}

// y <- (r p - r q) x + b y with p, q device scalars (the loop of axpby_kernel with the coefficient formed on the
// device as the host forms it).
__global__ void axpby_diff_kernel(double r, const double* __restrict__ p, const double* __restrict__ q,
                                  const double* __restrict__ x, double b, double* __restrict__ y, int64_t n) {
  const double a = rounded_diff(r, p[0], q[0]);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * (double)x[i];
    if (b != 0.0) v += b * (double)y[i];
    y[i] = (double)v;
  }
}

template <typename T>
__global__ void scal_kernel(double a, T* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)(a * (double)x[i]);
}

template <typename TD, typename TS>
__global__ void copy_kernel(TD* __restrict__ d, const TS* __restrict__ s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (TD)s[i];
}

template <typename T>
__global__ void fill_kernel(T* x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)v;
}

// 32x32 tile pairs (I, J) with I <= J; each tile pair is symmetrised through LDS.
template <typename T>
__global__ void symmetrize_kernel(T* x, int64_t dim) {
  __shared__ T a[32][33], b[32][33];
  const int64_t ntile = (dim + 31) / 32;
  // map blockIdx.x to (I, J) with I <= J: the rows above I hold S(I) = I ntile - I (I - 1) / 2 pairs; I from the
  // root of that quadratic, corrected for rounding
  const int64_t t = blockIdx.x;
  auto S = [ntile](int64_t r) { return r * ntile - r * (r - 1) / 2; };
  const double nn = 2.0 * (double)ntile + 1.0;
  int64_t I = (int64_t)((nn - sqrt(nn * nn - 8.0 * (double)t)) * 0.5);
  if (I < 0) I = 0;
  while (I + 1 <= ntile && S(I + 1) <= t) ++I;
  while (I > 0 && S(I) > t) --I;
  const int64_t J = I + (t - S(I));
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int r = ty; r < 32; r += 8) {
    int64_t i = I * 32 + r, j = J * 32 + tx;
    a[r][tx] = (i < dim && j < dim) ? x[i * dim + j] : T(0);
    int64_t i2 = J * 32 + r, j2 = I * 32 + tx;
    b[r][tx] = (i2 < dim && j2 < dim) ? x[i2 * dim + j2] : T(0);
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int64_t i = I * 32 + r, j = J * 32 + tx;
    T v = T(0.5) * (a[r][tx] + b[tx][r]);
    if (i < dim && j < dim) x[i * dim + j] = v;
    int64_t i2 = J * 32 + r, j2 = I * 32 + tx;
    T w = T(0.5) * (b[r][tx] + a[tx][r]);
    if (i2 < dim && j2 < dim && I != J) x[i2 * dim + j2] = w;
  }
}

template <typename T>
__global__ void add_diag_kernel(T* x, int64_t dim, double c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += (int64_t)gridDim.x * blockDim.x)
    x[i * dim + i] = (T)((double)x[i * dim + i] + c);
}

template <typename T>
__global__ void trace_kernel(const T* x, int64_t dim, double* out) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)x[i * dim + i];
  block_sum_store(s, out);
}

int grid_for(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

double finish_partials(Ctx& ctx, int blocks) {
  double host[RED_BLOCKS];
  MERA_HIP(hipMemcpyAsync(host, ctx.red.ptr, blocks * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();
  double s = 0.0;
  for (int i = 0; i < blocks; ++i) s += host[i];
  return s;
}

// ---- Jacobi --------------------------------------------------------------------------------------------

// Rotation of one tournament pair (i, j) that zeroes A_ij of the 2x2 block (Golub & Van Loan's symmetric
// Schur step); a dummy partner (-1, odd dimension) gives the identity.
__device__ inline void rot_of(const double* a, int dim, int i, int j, double& c, double& s) {
  if (i < 0 || j < 0) { c = 1.0; s = 0.0; return; }
  const double aii = a[(int64_t)i * dim + i], ajj = a[(int64_t)j * dim + j], aij = a[(int64_t)i * dim + j];
  if (aij == 0.0) { c = 1.0; s = 0.0; return; }
  const double tau = (ajj - aii) / (2.0 * aij);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// One round: every index is in exactly one pair; A' = J^T A J block by block (P, Q) of 2x2 entries, reading
// ain and writing aout; V <- V J in place. pairs: npairs x 2 ints for this round (-1 = dummy).
__global__ void jacobi_round_kernel(const double* __restrict__ ain, double* __restrict__ aout, double* v,
                                    const int* __restrict__ pairs, int npairs, int dim) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nblk = (int64_t)npairs * npairs;
  if (id < nblk) {
    const int P = (int)(id / npairs), Q = (int)(id % npairs);
    const int i = pairs[2 * P], j = pairs[2 * P + 1], k = pairs[2 * Q], l = pairs[2 * Q + 1];
    double cp, sp, cq, sq;
    rot_of(ain, dim, i, j, cp, sp);
    rot_of(ain, dim, k, l, cq, sq);
    // entries (row in {i,j}) x (col in {k,l}); a missing index (dummy) contributes nothing
    double aik = (i >= 0 && k >= 0) ? ain[(int64_t)i * dim + k] : 0.0;
    double ail = (i >= 0 && l >= 0) ? ain[(int64_t)i * dim + l] : 0.0;
    double ajk = (j >= 0 && k >= 0) ? ain[(int64_t)j * dim + k] : 0.0;
    double ajl = (j >= 0 && l >= 0) ? ain[(int64_t)j * dim + l] : 0.0;
    // T = J_P^T A_PQ
    double t0k = cp * aik - sp * ajk, t0l = cp * ail - sp * ajl;
    double t1k = sp * aik + cp * ajk, t1l = sp * ail + cp * ajl;
    // A' = T J_Q
    double n_ik = cq * t0k - sq * t0l, n_il = sq * t0k + cq * t0l;
    double n_jk = cq * t1k - sq * t1l, n_jl = sq * t1k + cq * t1l;
    if (P == Q) { n_il = 0.0; n_jk = 0.0; }
    if (i >= 0 && k >= 0) aout[(int64_t)i * dim + k] = n_ik;
    if (i >= 0 && l >= 0) aout[(int64_t)i * dim + l] = n_il;
    if (j >= 0 && k >= 0) aout[(int64_t)j * dim + k] = n_jk;
    if (j >= 0 && l >= 0) aout[(int64_t)j * dim + l] = n_jl;
  }
  // V <- V J: thread -> (row r, pair P)
  const int64_t nv = (int64_t)dim * npairs;
  if (id < nv) {
    const int r = (int)(id / npairs), P = (int)(id % npairs);
    const int i = pairs[2 * P], j = pairs[2 * P + 1];
    if (i >= 0 && j >= 0) {
      double cp, sp;
      rot_of(ain, dim, i, j, cp, sp);
      const double vi = v[(int64_t)r * dim + i], vj = v[(int64_t)r * dim + j];
      v[(int64_t)r * dim + i] = cp * vi - sp * vj;
      v[(int64_t)r * dim + j] = sp * vi + cp * vj;
    }
  }
}

// Matrices up to this size are decomposed by one workgroup, with A and V in LDS and every sweep in one launch.
constexpr int kJacobiSmall = 64;

// One decomposition of a batch launch (one workgroup each).
struct JacobiSmallTask {
  double* a;
  double* lam;
  double* v;
  const int* pairs;
  double tol;
  int npairs, rounds, dim, max_sweeps, v_init;
};
constexpr int kJacobiBatch = 16;
struct JacobiSmallBatch {
  JacobiSmallTask t[kJacobiBatch];
};

// The same rounds and stopping rule as the multi-launch path, for dim <= kJacobiSmall, one matrix per workgroup
// (workgroup b decomposes task b of the batch): per round the rotations of all pairs are taken from A, the 2x2
// blocks of J^T A J are formed in registers (at most 4 blocks per thread) and written back after a barrier, and
// V <- V J in place (each (row, pair) belongs to one thread).
__global__ void __launch_bounds__(256) jacobi_small_kernel(JacobiSmallBatch batch) {
  const JacobiSmallTask& task = batch.t[blockIdx.x];
  double* const a = task.a;
  double* const lam = task.lam;
  double* const v = task.v;
  const int* __restrict__ pairs = task.pairs;
  const int npairs = task.npairs, rounds = task.rounds, dim = task.dim, max_sweeps = task.max_sweeps;
  const int v_init = task.v_init;
  const double tol = task.tol;
  constexpr int LD = kJacobiSmall + 1;
  constexpr int NB = (kJacobiSmall / 2) * (kJacobiSmall / 2) / 256;
  __shared__ double As[kJacobiSmall * LD], Vs[kJacobiSmall * LD];
  __shared__ double cs[kJacobiSmall / 2], sn[kJacobiSmall / 2];
  __shared__ double part[4];
  const int tid = threadIdx.x;
  const int n2 = dim * dim;
  for (int t = tid; t < n2; t += 256) {
    const int r = t / dim, c = t - r * dim;
    As[r * LD + c] = a[t];
    Vs[r * LD + c] = v_init ? v[t] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  auto block_sum = [&](double x) {
    x = wave_sum(x);
    if ((tid & 63) == 0) part[tid >> 6] = x;
    __syncthreads();
    const double tot = part[0] + part[1] + part[2] + part[3];
    __syncthreads();
    return tot;
  };
  double f2 = 0.0;
  for (int t = tid; t < n2; t += 256) {
    const double x = As[(t / dim) * LD + t % dim];
    f2 += x * x;
  }
  const double fro = sqrt(block_sum(f2));
  double prev_off = INFINITY;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double o2 = 0.0;
    for (int t = tid; t < n2; t += 256) {
      const int r = t / dim, c = t - r * dim;
      if (r != c) o2 += As[r * LD + c] * As[r * LD + c];
    }
    const double off = sqrt(block_sum(o2));
    if (!(off > tol * fro) || dim == 1) break;
    if (sweep >= 4 && off > 0.25 * prev_off && off < 1e-12 * fro) break;
    prev_off = off;
    for (int rd = 0; rd < rounds; ++rd) {
      const int* pr = pairs + (size_t)rd * npairs * 2;
      if (tid < npairs) {
        double c, s;
        rot_of(As, LD, pr[2 * tid], pr[2 * tid + 1], c, s);
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      double nv[NB][4];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int id = tid + q * 256;
        if (id < npairs * npairs) {
          const int P = id / npairs, Q = id - P * npairs;
          const int i = pr[2 * P], j = pr[2 * P + 1], k = pr[2 * Q], l = pr[2 * Q + 1];
          const double cp = cs[P], sp = sn[P], cq = cs[Q], sq = sn[Q];
          const double aik = (i >= 0 && k >= 0) ? As[i * LD + k] : 0.0;
          const double ail = (i >= 0 && l >= 0) ? As[i * LD + l] : 0.0;
          const double ajk = (j >= 0 && k >= 0) ? As[j * LD + k] : 0.0;
          const double ajl = (j >= 0 && l >= 0) ? As[j * LD + l] : 0.0;
          const double t0k = cp * aik - sp * ajk, t0l = cp * ail - sp * ajl;
          const double t1k = sp * aik + cp * ajk, t1l = sp * ail + cp * ajl;
          nv[q][0] = cq * t0k - sq * t0l;
          nv[q][1] = (P == Q) ? 0.0 : sq * t0k + cq * t0l;
          nv[q][2] = (P == Q) ? 0.0 : cq * t1k - sq * t1l;
          nv[q][3] = sq * t1k + cq * t1l;
        }
      }
      for (int id = tid; id < dim * npairs; id += 256) {
        const int r = id / npairs, P = id - r * npairs;
        const int i = pr[2 * P], j = pr[2 * P + 1];
        if (i >= 0 && j >= 0) {
          const double vi = Vs[r * LD + i], vj = Vs[r * LD + j];
          Vs[r * LD + i] = cs[P] * vi - sn[P] * vj;
          Vs[r * LD + j] = sn[P] * vi + cs[P] * vj;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int id = tid + q * 256;
        if (id < npairs * npairs) {
          const int P = id / npairs, Q = id - P * npairs;
          const int i = pr[2 * P], j = pr[2 * P + 1], k = pr[2 * Q], l = pr[2 * Q + 1];
          if (i >= 0 && k >= 0) As[i * LD + k] = nv[q][0];
          if (i >= 0 && l >= 0) As[i * LD + l] = nv[q][1];
          if (j >= 0 && k >= 0) As[j * LD + k] = nv[q][2];
          if (j >= 0 && l >= 0) As[j * LD + l] = nv[q][3];
        }
      }
      __syncthreads();
    }
  }
  for (int t = tid; t < dim; t += 256) lam[t] = As[t * LD + t];
  for (int t = tid; t < n2; t += 256) {
    const int r = t / dim, c = t - r * dim;
    a[t] = As[r * LD + c];
    v[t] = Vs[r * LD + c];
  }
}

// Matrices above kJacobiSmall and up to this size are decomposed by one workgroup of kMidThreads threads each, A
// (ping-pong) and V in global memory (L2-resident at these sizes), every sweep in one launch: no launch per round
// and no host synchronisation per sweep, and the matrices of one batch run side by side. A round's work grows
// as dim^2 on one workgroup, so above this size the per-round launches over the whole GPU are faster.
constexpr int kJacobiMid = 160;
constexpr int kMidThreads = 1024;

struct JacobiMidTask {
  double* a;  // in: the matrix; out: the rotated matrix (diagonal = eigenvalues)
  double* b;  // ping-pong buffer, dim x dim
  double* lam;
  double* v;
  const int* pairs;
  double tol;
  int npairs, rounds, dim, max_sweeps, v_init;
};
struct JacobiMidBatch {
  JacobiMidTask t[kJacobiBatch];
};

// The rounds, rotations and block updates of jacobi_round_kernel, and the stopping rule of the multi-launch path
// (off-diagonal and Frobenius norms summed in the workgroup), with a barrier between rounds.
__global__ void __launch_bounds__(kMidThreads) jacobi_mid_kernel(JacobiMidBatch batch) {
  const JacobiMidTask& task = batch.t[blockIdx.x];
  const int dim = task.dim, npairs = task.npairs, rounds = task.rounds;
  const int* __restrict__ pairs = task.pairs;
  double* const v = task.v;
  __shared__ double cs[kJacobiMid / 2], sn[kJacobiMid / 2];
  __shared__ double part[kMidThreads / 64];
  const int tid = threadIdx.x;
  const int64_t n2 = (int64_t)dim * dim;
  auto block_sum = [&](double x) {
    x = wave_sum(x);
    if ((tid & 63) == 0) part[tid >> 6] = x;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < kMidThreads / 64; ++w) tot += part[w];
    __syncthreads();
    return tot;
  };
  if (!task.v_init)
    for (int64_t t = tid; t < n2; t += kMidThreads) v[t] = (t / dim == t % dim) ? 1.0 : 0.0;
  double* cur = task.a;
  double* nxt = task.b;
  double f2 = 0.0;
  for (int64_t t = tid; t < n2; t += kMidThreads) f2 += cur[t] * cur[t];
  const double fro = sqrt(block_sum(f2));
  double prev_off = INFINITY;
  for (int sweep = 0; sweep < task.max_sweeps; ++sweep) {
    double o2 = 0.0;
    for (int64_t t = tid; t < n2; t += kMidThreads)
      if (t / dim != t % dim) o2 += cur[t] * cur[t];
    const double off = sqrt(block_sum(o2));
    if (!(off > task.tol * fro) || dim == 1) break;
    // rounding floor: off-diagonal mass no longer shrinks quadratically
    if (sweep >= 4 && off > 0.25 * prev_off && off < 1e-12 * fro) break;
    prev_off = off;
    for (int rd = 0; rd < rounds; ++rd) {
      const int* pr = pairs + (size_t)rd * npairs * 2;
      if (tid < npairs) {
        double c, s;
        rot_of(cur, dim, pr[2 * tid], pr[2 * tid + 1], c, s);
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      for (int id = tid; id < npairs * npairs; id += kMidThreads) {
        const int P = id / npairs, Q = id - P * npairs;
        const int i = pr[2 * P], j = pr[2 * P + 1], k = pr[2 * Q], l = pr[2 * Q + 1];
        const double cp = cs[P], sp = sn[P], cq = cs[Q], sq = sn[Q];
        double aik = (i >= 0 && k >= 0) ? cur[(int64_t)i * dim + k] : 0.0;
        double ail = (i >= 0 && l >= 0) ? cur[(int64_t)i * dim + l] : 0.0;
        double ajk = (j >= 0 && k >= 0) ? cur[(int64_t)j * dim + k] : 0.0;
        double ajl = (j >= 0 && l >= 0) ? cur[(int64_t)j * dim + l] : 0.0;
        double t0k = cp * aik - sp * ajk, t0l = cp * ail - sp * ajl;
        double t1k = sp * aik + cp * ajk, t1l = sp * ail + cp * ajl;
        double n_ik = cq * t0k - sq * t0l, n_il = sq * t0k + cq * t0l;
        double n_jk = cq * t1k - sq * t1l, n_jl = sq * t1k + cq * t1l;
        if (P == Q) { n_il = 0.0; n_jk = 0.0; }
        if (i >= 0 && k >= 0) nxt[(int64_t)i * dim + k] = n_ik;
        if (i >= 0 && l >= 0) nxt[(int64_t)i * dim + l] = n_il;
        if (j >= 0 && k >= 0) nxt[(int64_t)j * dim + k] = n_jk;
        if (j >= 0 && l >= 0) nxt[(int64_t)j * dim + l] = n_jl;
      }
      for (int id = tid; id < dim * npairs; id += kMidThreads) {
        const int r = id / npairs, P = id - r * npairs;
        const int i = pr[2 * P], j = pr[2 * P + 1];
        if (i >= 0 && j >= 0) {
          const double cp = cs[P], sp = sn[P];
          const double vi = v[(int64_t)r * dim + i], vj = v[(int64_t)r * dim + j];
          v[(int64_t)r * dim + i] = cp * vi - sp * vj;
          v[(int64_t)r * dim + j] = sp * vi + cp * vj;
        }
      }
      __syncthreads();
      double* t = cur;
      cur = nxt;
      nxt = t;
    }
  }
  for (int t = tid; t < dim; t += kMidThreads) task.lam[t] = cur[(int64_t)t * dim + t];
  if (cur != task.a)
    for (int64_t t = tid; t < n2; t += kMidThreads) task.a[t] = cur[t];
}

__global__ void offdiag_kernel(const double* a, int dim, double* out) {
  double s = 0.0;
  const int64_t n = (int64_t)dim * dim;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / dim, j = t - i * dim;
    double x = a[t];
    if (i != j) s += x * x;
  }
  block_sum_store(s, out);
}

__global__ void diag_kernel(const double* a, int dim, double* lam) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < dim) lam[i] = a[(int64_t)i * dim + i];
}

__global__ void eye_kernel(double* v, int dim) {
  const int64_t n = (int64_t)dim * dim;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / dim, j = t - i * dim;
    v[t] = (i == j) ? 1.0 : 0.0;
  }
}

__global__ void scale_sylvester_kernel(double* m, const double* f, int dim) {
  const int64_t n = (int64_t)dim * dim;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / dim, j = t - i * dim;
    m[t] = m[t] * 2.0 / (f[i] + f[j]);
  }
}

__global__ void scale_cols_kernel(double* m, const double* s, int64_t rows, int cols) {
  const int64_t n = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    m[t] *= s[t % cols];
}

__global__ void copy_block_kernel(double* dst, int64_t ldd, const double* src, int64_t lds, int rows, int cols,
                                  double a) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / cols, j = t - i * cols;
    dst[i * ldd + j] = a * src[i * lds + j];
  }
}

// rho1[i, j] = ( sum_k rho[(i k), (j k)] + sum_k rho[(k i), (k j)] ) / 2 for a two-site rho (b^2 x b^2, FP64)
__global__ void marginal_pair_kernel(const double* __restrict__ rho, int b, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= b * b) return;
  const int i = t / b, j = t - i * b;
  const int64_t n = (int64_t)b * b;
  double s = 0.0;
  for (int k = 0; k < b; ++k) s += rho[(int64_t)(i * b + k) * n + (j * b + k)] + rho[(int64_t)(k * b + i) * n + (k * b + j)];
  out[t] = 0.5 * s;
}

__global__ void reg_spectrum_kernel(const double* lam, double delta, double* f, double* g, int dim) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < dim) {
    double x = sqrt(lam[i] * lam[i] + delta * delta);
    f[i] = x;
    g[i] = 1.0 / x;
  }
}

template <typename T>
__global__ void marginal2_kernel(const T* __restrict__ rho, int b, double* __restrict__ out) {
  const int64_t b2 = (int64_t)b * b, b3 = b2 * b, n = b2 * b2;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = t / (b * b2), y = (t / b2) % b, X = (t / b) % b, Y = t % b;
    double s = 0.0;
    for (int r = 0; r < b; ++r) s += (double)rho[((x * b + y) * b + r) * b3 + (X * b + Y) * b + r];
    for (int p = 0; p < b; ++p) s += (double)rho[((p * b + x) * b + y) * b3 + (p * b + X) * b + Y];
    out[t] = 0.5 * s;
  }
}

template <typename T>
__global__ void marginal1_kernel(const T* __restrict__ rho, int b, double* __restrict__ out) {
  const int64_t b3 = (int64_t)b * b * b;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < b * b) {
    const int q = t / b, Q = t % b;
    double s = 0.0;
    for (int p = 0; p < b; ++p)
      for (int r = 0; r < b; ++r) s += (double)rho[((int64_t)(p * b + q) * b + r) * b3 + (p * b + Q) * b + r];
    out[t] = s;
  }
}

struct JacobiSchedule {
  int dim = 0, npairs = 0, rounds = 0;
  DevBuf pairs;  // rounds x npairs x 2
};

}  // namespace

namespace {

// Launches the partial sums of <x, y> into out[0 .. blocks) and returns the block count.
int dot_launch(Ctx& ctx, VPtr x, VPtr y, int64_t n, double* out) {
  const int blocks = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (n + TPB - 1) / TPB));
  if (x.dbl() && y.dbl())
    hipLaunchKernelGGL((dot_kernel<double, double>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const double*)x.p, (const double*)y.p, n, out);
  else if (x.dbl())
    hipLaunchKernelGGL((dot_kernel<double, float>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const double*)x.p, (const float*)y.p, n, out);
  else if (y.dbl())
    hipLaunchKernelGGL((dot_kernel<float, double>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const float*)x.p, (const double*)y.p, n, out);
  else
    hipLaunchKernelGGL((dot_kernel<float, float>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const float*)x.p, (const float*)y.p, n, out);
  MERA_HIP(hipGetLastError());
  return blocks;
}

}  // namespace

void dots(Ctx& ctx, const VPtr* x, const VPtr* y, const int64_t* n, int count, double* out) {
  if (count <= 0) return;
  ctx.red.ensure((size_t)count * RED_BLOCKS * sizeof(double));
  double* part = ctx.red.as<double>();
  std::vector<int> blocks(count);
  int64_t total = 0;
  for (int i = 0; i < count; ++i) {
    blocks[i] = dot_launch(ctx, x[i], y[i], n[i], part + total);
    total += blocks[i];
  }
  std::vector<double> host((size_t)total);
  MERA_HIP(hipMemcpyAsync(host.data(), part, (size_t)total * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();
  // each product summed over its partials in order, as dot() does
  int64_t o = 0;
  for (int i = 0; i < count; ++i) {
    double s = 0.0;
    for (int b = 0; b < blocks[i]; ++b) s += host[(size_t)(o + b)];
    out[i] = s;
    o += blocks[i];
  }
}

double dot(Ctx& ctx, VPtr x, VPtr y, int64_t n) {
  ctx.red.ensure(RED_BLOCKS * sizeof(double));
  int blocks = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (n + TPB - 1) / TPB));
  double* out = ctx.red.as<double>();
  if (x.dbl() && y.dbl())
    hipLaunchKernelGGL((dot_kernel<double, double>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const double*)x.p, (const double*)y.p, n, out);
  else if (x.dbl())
    hipLaunchKernelGGL((dot_kernel<double, float>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const double*)x.p, (const float*)y.p, n, out);
  else if (y.dbl())
    hipLaunchKernelGGL((dot_kernel<float, double>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const float*)x.p, (const double*)y.p, n, out);
  else
    hipLaunchKernelGGL((dot_kernel<float, float>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const float*)x.p, (const float*)y.p, n, out);
  MERA_HIP(hipGetLastError());
  return finish_partials(ctx, blocks);
}

double nrm2(Ctx& ctx, VPtr x, int64_t n) { return std::sqrt(dot(ctx, x, x, n)); }

void multi_dot(Ctx& ctx, const VPtr* v, int k, VPtr w, int64_t n, double* out) {
  for (int j = 0; j < k; ++j)
    MERA_CHECK(v[j].dbl() == w.dbl(), MERA_EINVAL, "multi_dot: vectors of different precisions");
  const int blocks = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (n + TPB - 1) / TPB));
  ctx.red.ensure(((size_t)kMulti * blocks + kMulti) * sizeof(double));
  double* part = ctx.red.as<double>();
  double* sums = part + (size_t)kMulti * blocks;
  for (int j0 = 0; j0 < k; j0 += kMulti) {
    const int kk = std::min(kMulti, k - j0);
    if (w.dbl())
      hipLaunchKernelGGL(multi_dot_kernel<double>, dim3(blocks), dim3(TPB), 0, ctx.stream,
                         vec_list<double>(v + j0, nullptr, kk), kk, (const double*)w.p, n, part);
    else
      hipLaunchKernelGGL(multi_dot_kernel<float>, dim3(blocks), dim3(TPB), 0, ctx.stream,
                         vec_list<float>(v + j0, nullptr, kk), kk, (const float*)w.p, n, part);
    MERA_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_partials_kernel, dim3(kk), dim3(64), 0, ctx.stream, (const double*)part, blocks, sums);
    MERA_HIP(hipGetLastError());
    MERA_HIP(hipMemcpyAsync(out + j0, sums, kk * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    ctx.sync();
  }
}

void multi_axpby(Ctx& ctx, const VPtr* v, const double* c, int k, double b, VPtr y, int64_t n) {
  for (int j = 0; j < k; ++j) {
    MERA_CHECK(v[j].dbl() == y.dbl(), MERA_EINVAL, "multi_axpby: vectors of different precisions");
    MERA_CHECK(v[j].p != y.p, MERA_EINVAL, "multi_axpby: output aliases an input");
  }
  if (k == 0) {
    if (b == 0.0) fill(ctx, y, n, 0.0);
    else if (b != 1.0) scal(ctx, b, y, n);
    return;
  }
  const int g = grid_for(n);
  for (int j0 = 0; j0 < k; j0 += kMulti) {
    const int kk = std::min(kMulti, k - j0);
    const double bb = j0 == 0 ? b : 1.0;
    if (y.dbl())
      hipLaunchKernelGGL(multi_axpby_kernel<double>, dim3(g), dim3(TPB), 0, ctx.stream,
                         vec_list<double>(v + j0, c + j0, kk), kk, bb, (double*)y.p, n);
    else
      hipLaunchKernelGGL(multi_axpby_kernel<float>, dim3(g), dim3(TPB), 0, ctx.stream,
                         vec_list<float>(v + j0, c + j0, kk), kk, bb, (float*)y.p, n);
    MERA_HIP(hipGetLastError());
  }
}

void axpby(Ctx& ctx, double a, VPtr x, double b, VPtr y, int64_t n) {
  int g = grid_for(n);
  if (x.dbl() && y.dbl())
    hipLaunchKernelGGL((axpby_kernel<double, double>), dim3(g), dim3(TPB), 0, ctx.stream, a, (const double*)x.p, b,
                       (double*)y.p, n);
  else if (x.dbl())
    hipLaunchKernelGGL((axpby_kernel<double, float>), dim3(g), dim3(TPB), 0, ctx.stream, a, (const double*)x.p, b,
                       (float*)y.p, n);
  else if (y.dbl())
    hipLaunchKernelGGL((axpby_kernel<float, double>), dim3(g), dim3(TPB), 0, ctx.stream, a, (const float*)x.p, b,
                       (double*)y.p, n);
  else
    hipLaunchKernelGGL((axpby_kernel<float, float>), dim3(g), dim3(TPB), 0, ctx.stream, a, (const float*)x.p, b,
                       (float*)y.p, n);
  MERA_HIP(hipGetLastError());
}

void scal(Ctx& ctx, double a, VPtr x, int64_t n) {
  int g = grid_for(n);
  if (x.dbl()) hipLaunchKernelGGL(scal_kernel<double>, dim3(g), dim3(TPB), 0, ctx.stream, a, (double*)x.p, n);
  else hipLaunchKernelGGL(scal_kernel<float>, dim3(g), dim3(TPB), 0, ctx.stream, a, (float*)x.p, n);
  MERA_HIP(hipGetLastError());
}

void copy(Ctx& ctx, VPtr d, VPtr s, int64_t n) {
  if (n <= 0) return;
  if (d.dbl() == s.dbl()) {
    MERA_HIP(hipMemcpyAsync(d.p, s.p, n * (d.dbl() ? 8 : 4), hipMemcpyDeviceToDevice, ctx.stream));
    return;
  }
  int g = grid_for(n);
  if (d.dbl())
    hipLaunchKernelGGL((copy_kernel<double, float>), dim3(g), dim3(TPB), 0, ctx.stream, (double*)d.p,
                       (const float*)s.p, n);
  else
    hipLaunchKernelGGL((copy_kernel<float, double>), dim3(g), dim3(TPB), 0, ctx.stream, (float*)d.p,
                       (const double*)s.p, n);
  MERA_HIP(hipGetLastError());
}

void fill(Ctx& ctx, VPtr x, int64_t n, double v) {
  int g = grid_for(n);
  if (x.dbl()) hipLaunchKernelGGL(fill_kernel<double>, dim3(g), dim3(TPB), 0, ctx.stream, (double*)x.p, n, v);
  else hipLaunchKernelGGL(fill_kernel<float>, dim3(g), dim3(TPB), 0, ctx.stream, (float*)x.p, n, v);
  MERA_HIP(hipGetLastError());
}

void symmetrize(Ctx& ctx, VPtr x, int64_t dim) {
  const int64_t nt = (dim + 31) / 32;
  const int64_t blocks = nt * (nt + 1) / 2;
  if (x.dbl())
    hipLaunchKernelGGL(symmetrize_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, ctx.stream, (double*)x.p,
                       dim);
  else
    hipLaunchKernelGGL(symmetrize_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, ctx.stream, (float*)x.p,
                       dim);
  MERA_HIP(hipGetLastError());
}

void add_diag(Ctx& ctx, VPtr x, int64_t dim, double c) {
  int g = grid_for(dim);
  if (x.dbl()) hipLaunchKernelGGL(add_diag_kernel<double>, dim3(g), dim3(TPB), 0, ctx.stream, (double*)x.p, dim, c);
  else hipLaunchKernelGGL(add_diag_kernel<float>, dim3(g), dim3(TPB), 0, ctx.stream, (float*)x.p, dim, c);
  MERA_HIP(hipGetLastError());
}

double trace(Ctx& ctx, VPtr x, int64_t dim) {
  ctx.red.ensure(RED_BLOCKS * sizeof(double));
  int blocks = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (dim + TPB - 1) / TPB));
  if (x.dbl())
    hipLaunchKernelGGL(trace_kernel<double>, dim3(blocks), dim3(TPB), 0, ctx.stream, (const double*)x.p, dim,
                       ctx.red.as<double>());
  else
    hipLaunchKernelGGL(trace_kernel<float>, dim3(blocks), dim3(TPB), 0, ctx.stream, (const float*)x.p, dim,
                       ctx.red.as<double>());
  MERA_HIP(hipGetLastError());
  return finish_partials(ctx, blocks);
}

// ---- device-resident scalars ----------------------------------------------------------------------------

void dot_dev(Ctx& ctx, VPtr x, VPtr y, int64_t n, double* out_dev) {
  ctx.red.ensure(RED_BLOCKS * sizeof(double));
  const int blocks = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (n + TPB - 1) / TPB));
  double* part = ctx.red.as<double>();
  if (x.dbl() && y.dbl())
    hipLaunchKernelGGL((dot_kernel<double, double>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const double*)x.p, (const double*)y.p, n, part);
  else if (x.dbl())
    hipLaunchKernelGGL((dot_kernel<double, float>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const double*)x.p, (const float*)y.p, n, part);
  else if (y.dbl())
    hipLaunchKernelGGL((dot_kernel<float, double>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const float*)x.p, (const double*)y.p, n, part);
  else
    hipLaunchKernelGGL((dot_kernel<float, float>), dim3(blocks), dim3(TPB), 0, ctx.stream,
                       (const float*)x.p, (const float*)y.p, n, part);
  MERA_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, ctx.stream, (const double*)part, blocks, out_dev);
  MERA_HIP(hipGetLastError());
}

void dot_dev_exact(Ctx& ctx, const double* x, const double* y, int64_t n, double* out_dev) {
  ctx.red.ensure(RED_BLOCKS * sizeof(double));
  double* part = ctx.red.as<double>();
  const int blocks = dot_launch(ctx, VPtr{(void*)x, Prec::F64}, VPtr{(void*)y, Prec::F64}, n, part);
  hipLaunchKernelGGL(sum_partials_seq_kernel, dim3(1), dim3(64), 0, ctx.stream, (const double*)part, blocks, out_dev);
  MERA_HIP(hipGetLastError());
}

void scal_ratio_dev(Ctx& ctx, const double* num_dev, const double* den_dev, double* x, int64_t n) {
  hipLaunchKernelGGL(scal_ratio_kernel<double>, dim3(grid_for(n)), dim3(TPB), 0, ctx.stream, num_dev, den_dev, x, n);
  MERA_HIP(hipGetLastError());
}

void axpby_diff_dev(Ctx& ctx, double r, const double* p_dev, const double* q_dev, const double* x, double b,
                    double* y, int64_t n) {
  hipLaunchKernelGGL(axpby_diff_kernel, dim3(grid_for(n)), dim3(TPB), 0, ctx.stream, r, p_dev, q_dev, x, b, y, n);
  MERA_HIP(hipGetLastError());
}

void trace_dev(Ctx& ctx, VPtr x, int64_t dim, double* out_dev) {
  ctx.red.ensure(RED_BLOCKS * sizeof(double));
  const int blocks = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (dim + TPB - 1) / TPB));
  double* part = ctx.red.as<double>();
  if (x.dbl())
    hipLaunchKernelGGL(trace_kernel<double>, dim3(blocks), dim3(TPB), 0, ctx.stream, (const double*)x.p, dim, part);
  else
    hipLaunchKernelGGL(trace_kernel<float>, dim3(blocks), dim3(TPB), 0, ctx.stream, (const float*)x.p, dim, part);
  MERA_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, ctx.stream, (const double*)part, blocks, out_dev);
  MERA_HIP(hipGetLastError());
}

void axpby_dev(Ctx& ctx, const double* a_dev, double s, VPtr x, double b, VPtr y, int64_t n) {
  const int g = grid_for(n);
  if (x.dbl() && y.dbl())
    hipLaunchKernelGGL((axpby_dev_kernel<double, double>), dim3(g), dim3(TPB), 0, ctx.stream, a_dev, s,
                       (const double*)x.p, b, (double*)y.p, n);
  else if (x.dbl())
    hipLaunchKernelGGL((axpby_dev_kernel<double, float>), dim3(g), dim3(TPB), 0, ctx.stream, a_dev, s,
                       (const double*)x.p, b, (float*)y.p, n);
  else if (y.dbl())
    hipLaunchKernelGGL((axpby_dev_kernel<float, double>), dim3(g), dim3(TPB), 0, ctx.stream, a_dev, s,
                       (const float*)x.p, b, (double*)y.p, n);
  else
    hipLaunchKernelGGL((axpby_dev_kernel<float, float>), dim3(g), dim3(TPB), 0, ctx.stream, a_dev, s,
                       (const float*)x.p, b, (float*)y.p, n);
  MERA_HIP(hipGetLastError());
}

void add_diag_dev(Ctx& ctx, VPtr x, int64_t dim, const double* c_dev, double s) {
  const int g = grid_for(dim);
  if (x.dbl())
    hipLaunchKernelGGL(add_diag_dev_kernel<double>, dim3(g), dim3(TPB), 0, ctx.stream, (double*)x.p, dim, c_dev, s);
  else
    hipLaunchKernelGGL(add_diag_dev_kernel<float>, dim3(g), dim3(TPB), 0, ctx.stream, (float*)x.p, dim, c_dev, s);
  MERA_HIP(hipGetLastError());
}

void multi_dot_dev(Ctx& ctx, const VPtr* v, int k, VPtr w, int64_t n, double* out_dev) {
  for (int j = 0; j < k; ++j)
    MERA_CHECK(v[j].dbl() == w.dbl(), MERA_EINVAL, "multi_dot: vectors of different precisions");
  const int blocks = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (n + TPB - 1) / TPB));
  ctx.red.ensure((size_t)kMulti * blocks * sizeof(double));
  double* part = ctx.red.as<double>();
  for (int j0 = 0; j0 < k; j0 += kMulti) {
    const int kk = std::min(kMulti, k - j0);
    if (w.dbl())
      hipLaunchKernelGGL(multi_dot_kernel<double>, dim3(blocks), dim3(TPB), 0, ctx.stream,
                         vec_list<double>(v + j0, nullptr, kk), kk, (const double*)w.p, n, part);
    else
      hipLaunchKernelGGL(multi_dot_kernel<float>, dim3(blocks), dim3(TPB), 0, ctx.stream,
                         vec_list<float>(v + j0, nullptr, kk), kk, (const float*)w.p, n, part);
    MERA_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_partials_kernel, dim3(kk), dim3(64), 0, ctx.stream, (const double*)part, blocks,
                       out_dev + j0);
    MERA_HIP(hipGetLastError());
  }
}

void multi_axpby_dev(Ctx& ctx, const VPtr* v, const double* c_dev, double s, int k, double b, VPtr y, int64_t n) {
  for (int j = 0; j < k; ++j) {
    MERA_CHECK(v[j].dbl() == y.dbl(), MERA_EINVAL, "multi_axpby: vectors of different precisions");
    MERA_CHECK(v[j].p != y.p, MERA_EINVAL, "multi_axpby: output aliases an input");
  }
  const int g = grid_for(n);
  for (int j0 = 0; j0 < k; j0 += kMulti) {
    const int kk = std::min(kMulti, k - j0);
    const double bb = j0 == 0 ? b : 1.0;
    if (y.dbl())
      hipLaunchKernelGGL(multi_axpby_dev_kernel<double>, dim3(g), dim3(TPB), 0, ctx.stream,
                         vec_list<double>(v + j0, nullptr, kk), kk, c_dev + j0, s, bb, (double*)y.p, n);
    else
      hipLaunchKernelGGL(multi_axpby_dev_kernel<float>, dim3(g), dim3(TPB), 0, ctx.stream,
                         vec_list<float>(v + j0, nullptr, kk), kk, c_dev + j0, s, bb, (float*)y.p, n);
    MERA_HIP(hipGetLastError());
  }
}

void normalize_dev(Ctx& ctx, VPtr x, int64_t n, double* nrm_dev, double* work_dev) {
  dot_dev(ctx, x, x, n, work_dev);
  const int g = grid_for(n);
  if (x.dbl())
    hipLaunchKernelGGL(normalize_dev_kernel<double>, dim3(g), dim3(TPB), 0, ctx.stream, (double*)x.p, n,
                       (const double*)work_dev, nrm_dev);
  else
    hipLaunchKernelGGL(normalize_dev_kernel<float>, dim3(g), dim3(TPB), 0, ctx.stream, (float*)x.p, n,
                       (const double*)work_dev, nrm_dev);
  MERA_HIP(hipGetLastError());
}

namespace {

// Tournament (circle) schedule of the rounds for one dimension, built once per device and dimension: m = dim
// rounded up to even, index m - 1 a dummy when dim is odd.
JacobiSchedule& jacobi_schedule(Ctx& ctx, int dim) {
  static thread_local std::unordered_map<std::string, std::unique_ptr<JacobiSchedule>> scheds;
  const std::string key = std::to_string(ctx.device) + ":" + std::to_string(dim);
  auto it = scheds.find(key);
  if (it == scheds.end()) {
    auto s = std::make_unique<JacobiSchedule>();
    const int m = dim + (dim & 1);
    s->dim = dim;
    s->npairs = m / 2;
    s->rounds = m - 1;
    std::vector<int> host((size_t)s->rounds * s->npairs * 2);
    std::vector<int> ring(m);
    for (int i = 0; i < m; ++i) ring[i] = i;
    for (int r = 0; r < s->rounds; ++r) {
      for (int k = 0; k < s->npairs; ++k) {
        int i = ring[k], j = ring[m - 1 - k];
        host[((size_t)r * s->npairs + k) * 2] = (i < dim) ? i : -1;
        host[((size_t)r * s->npairs + k) * 2 + 1] = (j < dim) ? j : -1;
      }
      // rotate all but ring[0]
      int last = ring[m - 1];
      for (int i = m - 1; i > 1; --i) ring[i] = ring[i - 1];
      ring[1] = last;
    }
    s->pairs.alloc(host.size() * sizeof(int));
    MERA_HIP(hipMemcpyAsync(s->pairs.ptr, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice,
                            ctx.stream));
    MERA_HIP(hipStreamSynchronize(ctx.stream));
    it = scheds.emplace(key, std::move(s)).first;
  }
  return *it->second;
}

}  // namespace

// The multi-launch path (one kernel per round) for matrices above kJacobiMid.
void jacobi_eigh_rounds(Ctx& ctx, double* a, double* lam, double* v, int dim, double tol, int max_sweeps,
                        bool v_init);

void jacobi_eigh_batch(Ctx& ctx, const std::vector<JacobiTask>& tasks) {
  JacobiSmallBatch batch{};
  JacobiMidBatch mid{};
  int nb = 0, nm = 0;
  auto flush = [&]() {
    if (nb == 0) return;
    hipLaunchKernelGGL(jacobi_small_kernel, dim3(nb), dim3(256), 0, ctx.stream, batch);
    MERA_HIP(hipGetLastError());
    nb = 0;
  };
  auto flush_mid = [&]() {
    if (nm == 0) return;
    hipLaunchKernelGGL(jacobi_mid_kernel, dim3(nm), dim3(kMidThreads), 0, ctx.stream, mid);
    MERA_HIP(hipGetLastError());
    nm = 0;
  };
  for (const JacobiTask& t : tasks) {
    if (t.dim <= 0) continue;
    if (t.dim > kJacobiMid) {
      jacobi_eigh_rounds(ctx, t.a, t.lam, t.v, t.dim, t.tol, t.max_sweeps, t.v_init);
      continue;
    }
    JacobiSchedule& s = jacobi_schedule(ctx, t.dim);
    if (t.dim <= kJacobiSmall) {
      batch.t[nb++] = JacobiSmallTask{t.a, t.lam, t.v, s.pairs.as<int>(), t.tol, s.npairs, s.rounds, t.dim,
                                      t.max_sweeps, t.v_init ? 1 : 0};
      if (nb == kJacobiBatch) flush();
    } else {
      double* b = static_cast<double*>(ctx.buf("jacobi.mid" + std::to_string(nm),
                                               (size_t)t.dim * t.dim * sizeof(double)));
      mid.t[nm++] = JacobiMidTask{t.a, b, t.lam, t.v, s.pairs.as<int>(), t.tol, s.npairs, s.rounds, t.dim,
                                  t.max_sweeps, t.v_init ? 1 : 0};
      if (nm == kJacobiBatch) flush_mid();
    }
  }
  flush();
  flush_mid();
}

void jacobi_eigh(Ctx& ctx, double* a, double* lam, double* v, int dim, double tol, int max_sweeps, bool v_init) {
  if (dim <= 0) return;
  if (dim <= kJacobiMid) {
    jacobi_eigh_batch(ctx, {JacobiTask{a, lam, v, dim, tol, max_sweeps, v_init}});
    return;
  }
  jacobi_eigh_rounds(ctx, a, lam, v, dim, tol, max_sweeps, v_init);
}

void jacobi_eigh_rounds(Ctx& ctx, double* a, double* lam, double* v, int dim, double tol, int max_sweeps,
                        bool v_init) {
  JacobiSchedule& s = jacobi_schedule(ctx, dim);
  double* b = static_cast<double*>(ctx.buf("jacobi.pingpong", (size_t)dim * dim * sizeof(double)));
  const int g = grid_for((int64_t)dim * dim);
  if (!v_init) hipLaunchKernelGGL(eye_kernel, dim3(g), dim3(TPB), 0, ctx.stream, v, dim);
  const double fro = std::sqrt(dot(ctx, VPtr{a, Prec::F64}, VPtr{a, Prec::F64}, (int64_t)dim * dim));
  ctx.red.ensure(RED_BLOCKS * sizeof(double));
  const int64_t work = std::max<int64_t>((int64_t)s.npairs * s.npairs, (int64_t)dim * s.npairs);
  const int rg = (int)((work + TPB - 1) / TPB);
  int sweeps = 0;
  double* cur = a;
  double* nxt = b;
  double prev_off = INFINITY;
  for (; sweeps < max_sweeps; ++sweeps) {
    hipLaunchKernelGGL(offdiag_kernel, dim3(256), dim3(TPB), 0, ctx.stream, cur, dim, ctx.red.as<double>());
    double off = std::sqrt(finish_partials(ctx, 256));
    if (!(off > tol * fro) || dim == 1) break;
    // rounding floor: off-diagonal mass no longer shrinks quadratically
    if (sweeps >= 4 && off > 0.25 * prev_off && off < 1e-12 * fro) break;
    prev_off = off;
    for (int r = 0; r < s.rounds; ++r) {
      hipLaunchKernelGGL(jacobi_round_kernel, dim3(rg), dim3(TPB), 0, ctx.stream, cur, nxt, v,
                         s.pairs.as<int>() + (size_t)r * s.npairs * 2, s.npairs, dim);
      std::swap(cur, nxt);
    }
    MERA_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(diag_kernel, dim3((dim + TPB - 1) / TPB), dim3(TPB), 0, ctx.stream, cur, dim, lam);
  if (cur != a) MERA_HIP(hipMemcpyAsync(a, cur, (size_t)dim * dim * 8, hipMemcpyDeviceToDevice, ctx.stream));
  MERA_HIP(hipGetLastError());
}

void rho_marginals(Ctx& ctx, VPtr rho, int b, double* rho1, double* rho2) {
  const int64_t n2 = (int64_t)b * b * b * b;
  if (rho.dbl()) {
    hipLaunchKernelGGL(marginal2_kernel<double>, dim3(grid_for(n2)), dim3(TPB), 0, ctx.stream,
                       (const double*)rho.p, b, rho2);
    hipLaunchKernelGGL(marginal1_kernel<double>, dim3((b * b + TPB - 1) / TPB), dim3(TPB), 0, ctx.stream,
                       (const double*)rho.p, b, rho1);
  } else {
    hipLaunchKernelGGL(marginal2_kernel<float>, dim3(grid_for(n2)), dim3(TPB), 0, ctx.stream,
                       (const float*)rho.p, b, rho2);
    hipLaunchKernelGGL(marginal1_kernel<float>, dim3((b * b + TPB - 1) / TPB), dim3(TPB), 0, ctx.stream,
                       (const float*)rho.p, b, rho1);
  }
  MERA_HIP(hipGetLastError());
}

void scale_sylvester(Ctx& ctx, double* m, const double* f, int dim) {
  hipLaunchKernelGGL(scale_sylvester_kernel, dim3(grid_for((int64_t)dim * dim)), dim3(TPB), 0, ctx.stream, m, f,
                     dim);
  MERA_HIP(hipGetLastError());
}

void scale_cols(Ctx& ctx, double* m, const double* s, int64_t rows, int cols) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(rows * cols)), dim3(TPB), 0, ctx.stream, m, s, rows, cols);
  MERA_HIP(hipGetLastError());
}

void copy_block(Ctx& ctx, double* dst, int64_t ldd, const double* src, int64_t lds, int rows, int cols, double a) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(copy_block_kernel, dim3(grid_for((int64_t)rows * cols)), dim3(TPB), 0, ctx.stream, dst, ldd, src,
                     lds, rows, cols, a);
  MERA_HIP(hipGetLastError());
}

void rho_marginal_pair(Ctx& ctx, VPtr rho, int b, double* rho1) {
  MERA_CHECK(rho.dbl(), MERA_EINVAL, "rho_marginal_pair expects an FP64 matrix");
  hipLaunchKernelGGL(marginal_pair_kernel, dim3((b * b + TPB - 1) / TPB), dim3(TPB), 0, ctx.stream,
                     static_cast<const double*>(rho.p), b, rho1);
  MERA_HIP(hipGetLastError());
}

void reg_spectrum(Ctx& ctx, const double* lam, double delta, double* f, double* g, int dim) {
  hipLaunchKernelGGL(reg_spectrum_kernel, dim3((dim + TPB - 1) / TPB), dim3(TPB), 0, ctx.stream, lam, delta, f, g,
                     dim);
  MERA_HIP(hipGetLastError());
}

}  // namespace mera
