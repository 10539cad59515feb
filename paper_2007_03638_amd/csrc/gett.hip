// Permute-fused GETT kernels for gfx950: LDS-staged, register-prefetched tile loads (16-byte vectors where the
// layouts allow; row offsets from tables, k offsets computed from the contracted legs), MFMA inner products
// (f32 32x32x2, f64 16x16x4, bf16 16x16x32 for the split-bf16 form), split-K partials reduced in FP64.
#include "gett.h"

#include <algorithm>
#include <type_traits>

namespace mera {

namespace {

// One launch runs the same contraction (same tables and extents) for up to kGettMaxGroup independent operand
// sets; blockIdx.y selects the set.
struct Args {
  const void* A[kGettMaxGroup];
  const void* B[kGettMaxGroup];
  void* C[kGettMaxGroup];
  void* partial[kGettMaxGroup];  // splits x M x N partial sums per set (accumulator type); used when split != 0
  const int64_t* a_m;
  const int64_t* b_n;
  const int64_t* c_m;
  const int64_t* c_n;
  GettKLegs kl;
  int64_t M, N, K;
  int64_t kchunk;  // K range per split, a multiple of BK
  double alpha, beta;
  int split;       // 1: write partial sums, 0: write C
};

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Lane layouts (checked on gfx950 against a host GEMM):
//  f32 32x32x2:  A[m = lane%32][k = lane/32], B[k = lane/32][n = lane%32],
//                acc[i] -> row 8*(i/4) + 4*(lane/32) + i%4, col lane%32
//  f64 16x16x4:  A[m = lane%16][k = lane/16], B[k = lane/16][n = lane%16],
//                acc[i] -> row lane/16 + 4*i, col lane%16
//  bf16 16x16x32: A[m = lane%16][k = 8*(lane/16)+j], B[k = 8*(lane/16)+j][n = lane%16],
//                acc[i] -> row 4*(lane/16) + i, col lane%16
template <typename T> struct Mma;
template <> struct Mma<float> {
  static constexpr int MT = 32, NT = 32, KT = 2, NACC = 16;
  typedef f32x16 acc_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }
  __device__ static inline int col(int lane) { return lane & 31; }
};
template <> struct Mma<double> {
  static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4;
  typedef f64x4 acc_t;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return (lane >> 4) + 4 * i; }
  __device__ static inline int col(int lane) { return lane & 15; }
};

// Offset of the k-th index along the contracted legs (fastest leg first; see GettKLegs): NKL digit extractions
// by reciprocal multiplication, no memory access. Entries past kl.n are zero and contribute nothing.
template <int NKL>
__device__ inline uint64_t k_offset(uint32_t k, const GettKLegs& kl, const uint32_t* stride) {
  uint64_t off = 0;
  uint32_t q = k;
#pragma unroll
  for (int l = 0; l + 1 < NKL; ++l) {
    const uint32_t qn = __umulhi(q, kl.mag[l]);
    off += (uint64_t)(q - qn * kl.ext[l]) * stride[l];
    q = qn;
  }
  return off + (uint64_t)q * stride[NKL - 1];
}

// Tile loader: BMN x BK tile of an operand whose element (r, k) lives at base + off_r[r] + k_offset(k).
// KFAST: consecutive threads walk k (the operand's unit-stride leg is a K leg); each thread then owns one k
// and PER rows. Otherwise consecutive threads walk r in groups of 64; each thread owns NR rows and NK k's, and
// a wave's k's are the same for all its lanes, so their offsets are formed once per wave in scalar registers.
// Rows past the extent are not masked: their table entries are padded with offset 0, so they read a valid
// element and only feed accumulator rows that are never stored. k past the end of the range is clamped for the
// address and masked (zero) when the tile is staged, which only the last tile of a range needs (KMASK).
template <typename T, int BMN, int BK, bool KFAST, int NKL>
struct Loader {
  static constexpr int PER = BMN * BK / 256;
  static_assert(PER >= 1 && (BMN * BK) % 256 == 0, "tile too small for 256 threads");
  static_assert(KFAST ? (256 % BK == 0) : (BMN % 64 == 0), "thread mapping");
  static constexpr int NR = KFAST ? PER : BMN / 64;   // rows per thread
  static constexpr int NK = KFAST ? 1 : PER / NR;     // k's per thread
  static constexpr int RSTEP = KFAST ? 256 / BK : 64;
  static constexpr int KSTEP = KFAST ? 1 : 4;         // 256 threads / 64 rows per group
  static_assert(KFAST || NK * KSTEP == BK, "k coverage");
  const T* rowp[NR];
  int r0;
  uint32_t k0;
  T reg[PER];

  __device__ inline void init(const T* base, const int64_t* off_r, int64_t rbase, int tid) {
    if (KFAST) {
      k0 = tid % BK;
      r0 = tid / BK;
    } else {
      r0 = tid % 64;
      k0 = __builtin_amdgcn_readfirstlane(tid / 64);
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) rowp[i] = base + off_r[rbase + r0 + i * RSTEP];
  }
  // loads the tile starting at kt; element (i): row index i % NR, k index i / NR
  __device__ inline void load(int64_t kt, int64_t K, const GettKLegs& kl, const uint32_t* stride) {
    const uint32_t klast = (uint32_t)K - 1;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const uint32_t k = (uint32_t)kt + k0 + j * KSTEP;
      const uint64_t o = k_offset<NKL>(k < klast ? k : klast, kl, stride);
#pragma unroll
      for (int r = 0; r < NR; ++r) reg[j * NR + r] = rowp[r][o];
    }
  }
  // value of element i of the tile starting at kt, zero past kend when KMASK
  template <bool KMASK>
  __device__ inline T value(int i, int64_t kt, int64_t kend) const {
    return (KMASK && kt + k0 + (i / NR) * KSTEP >= kend) ? T(0) : reg[i];
  }
  __device__ inline int lds_index(int i, int LD) const {
    return (k0 + (i / NR) * KSTEP) * LD + r0 + (i % NR) * RSTEP;
  }
  // LDS tile stored k-major: lds[k * LD + r]
  template <int LD, bool KMASK>
  __device__ inline void store(T* lds, int64_t kt, int64_t kend) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) lds[lds_index(i, LD)] = value<KMASK>(i, kt, kend);
  }
  template <int LD>
  __device__ inline void store_tile(T* lds, int64_t kt, int64_t kend) const {
    if (kt + BK <= kend) store<LD, false>(lds, kt, kend);
    else store<LD, true>(lds, kt, kend);
  }
};

// Vectorised tile loader: each global load moves VW consecutive elements along the operand's unit-stride leg
// (VW = 4 for FP32, 2 for FP64: 16 bytes). Used when that leg is the fastest index the loader walks, its extent
// and every other stride are multiples of VW and the base is 16-byte aligned, so that every vector lies within
// one run of the unit-stride leg. KFAST: the vectors run along k (VW k's of one row; staged as VW scalar LDS
// writes); otherwise along rows (VW rows at one k; one vector LDS write). Vector i of a thread is the tile's
// vector number tid + 256 i; padded rows (offset 0) and clamped k read valid elements, as in Loader.
template <typename T, int BMN, int BK, bool KFAST, int NKL, int VW>
struct VecLoader {
  typedef T V __attribute__((ext_vector_type(VW)));
  static constexpr int G = KFAST ? BK / VW : BMN / VW;  // vectors along the walked dimension
  static constexpr int NV = BMN * BK / VW / 256;        // vectors per thread
  static_assert(NV >= 1 && (BMN * BK / VW) % 256 == 0, "tile too small for 256 threads");
  const T* rowp[NV];
  int rr[NV], kk[NV];
  V reg[NV];

  __device__ inline void init(const T* base, const int64_t* off_r, int64_t rbase, int tid) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = tid + 256 * i;
      rr[i] = KFAST ? e / G : (e % G) * VW;
      kk[i] = KFAST ? (e % G) * VW : e / G;
      rowp[i] = base + off_r[rbase + rr[i]];
    }
  }
  __device__ inline void load(int64_t kt, int64_t K, const GettKLegs& kl, const uint32_t* stride) {
    const uint32_t klast = (uint32_t)(KFAST ? K - VW : K - 1);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t k = (uint32_t)kt + (uint32_t)kk[i];
      const uint64_t o = k_offset<NKL>(k < klast ? k : klast, kl, stride);
      reg[i] = *reinterpret_cast<const V*>(rowp[i] + o);
    }
  }
  template <int LD, bool KMASK>
  __device__ inline void store(T* lds, int64_t kt, int64_t kend) const {
    static_assert(KFAST || LD % VW == 0, "vector LDS rows");
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (KFAST) {
#pragma unroll
        for (int j = 0; j < VW; ++j)
          lds[(kk[i] + j) * LD + rr[i]] = (KMASK && kt + kk[i] + j >= kend) ? T(0) : reg[i][j];
      } else {
        V v = reg[i];
        if (KMASK && kt + kk[i] >= kend) v = V(T(0));
        *reinterpret_cast<V*>(&lds[kk[i] * LD + rr[i]]) = v;
      }
    }
  }
  template <int LD>
  __device__ inline void store_tile(T* lds, int64_t kt, int64_t kend) const {
    if (kt + BK <= kend) store<LD, false>(lds, kt, kend);
    else store<LD, true>(lds, kt, kend);
  }
};

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on XCD b % 8). Remap so that each
// XCD processes a contiguous range of logical tiles: consecutive tiles share an A panel, which then stays in
// that XCD's L2 instead of being fetched by all eight. The tail (ntiles % 8 tiles) keeps the identity map.
__device__ inline int64_t xcd_tile(int64_t b, int64_t ntiles) {
  const int64_t full = ntiles / 8;
  return (b < full * 8) ? (b % 8) * full + b / 8 : b;
}

// Origin of logical tile `tile`. Tiles are taken in groups of kTileGroup panels of the dimension with more tiles
// (the larger operand); within a group that dimension runs fastest, then the other one. The 64 tiles an XCD runs
// at once then cover about 8 panels of each operand, which its L2 serves to all of them: each operand is fetched
// from beyond L2 about (tiles of the other dimension) / kTileGroup times instead of once per tile of the other
// dimension for the smaller operand.
constexpr int64_t kTileGroup = 8;
template <int BM, int BN>
__device__ inline void tile_origin(int64_t tile, int64_t M, int64_t N, int64_t& m0, int64_t& n0) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  const bool mgroups = tm >= tn;
  const int64_t tbig = mgroups ? tm : tn, tsmall = mgroups ? tn : tm;
  const int64_t grp = tile / (kTileGroup * tsmall), loc = tile % (kTileGroup * tsmall);
  const int64_t gsize = (tbig - grp * kTileGroup < kTileGroup) ? tbig - grp * kTileGroup : kTileGroup;
  const int64_t big = grp * kTileGroup + loc % gsize, small = loc / gsize;
  m0 = (mgroups ? big : small) * BM;
  n0 = (mgroups ? small : big) * BN;
}

template <typename T, int BM, int BN, int BK, bool AKF, bool BKF, int NKL, bool VEC>
// At most 256 registers per lane (2 waves per SIMD) for every tile; the register allocator then keeps the
// accumulators in VGPRs (the 128 x 64 FP64 tile fits in 168 and runs 3 waves per SIMD).
__global__ void __launch_bounds__(256, 2) gett_kernel(Args g) {
  using F = Mma<T>;
  // vector width of the tile loads (VEC: both operands qualify). LDS rows are padded: to a multiple of VW where
  // an operand is staged with vector writes (loads along rows), else by 2 FP32 / 1 FP64 elements, which keeps the
  // strided scalar writes of k-walking loads free of bank conflicts.
  constexpr int VW = VEC ? 16 / (int)sizeof(T) : 1;
  constexpr int PADS = sizeof(T) == 4 ? 2 : 1;
  constexpr int LDA = BM + ((VEC && !AKF) ? VW : PADS), LDB = BN + ((VEC && !BKF) ? VW : PADS);
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / F::MT, FN = WN / F::NT;
  static_assert(FM >= 1 && FN >= 1, "wave tile smaller than one MFMA block");
  __shared__ T As[2][BK * LDA];
  __shared__ T Bs[2][BK * LDB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * WM;
  const int wn = (wave & 1) * WN;

  int64_t m0, n0;
  tile_origin<BM, BN>(xcd_tile(blockIdx.x, gridDim.x), g.M, g.N, m0, n0);
  const int64_t kb = (int64_t)blockIdx.z * g.kchunk;
  const int64_t ke = (g.K < kb + g.kchunk) ? g.K : kb + g.kchunk;

  const int grp = blockIdx.y;
  const T* __restrict__ A = static_cast<const T*>(g.A[grp]);
  const T* __restrict__ B = static_cast<const T*>(g.B[grp]);

  std::conditional_t<VEC, VecLoader<T, BM, BK, AKF, NKL, VW>, Loader<T, BM, BK, AKF, NKL>> la;
  std::conditional_t<VEC, VecLoader<T, BN, BK, BKF, NKL, VW>, Loader<T, BN, BK, BKF, NKL>> lb;
  la.init(A, g.a_m, m0, tid);
  lb.init(B, g.b_n, n0, tid);

  typename F::acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < F::NACC; ++r) acc[i][j][r] = T(0);

  // MFMA operand fragments, double-buffered: the fragments of k-step s+1 are read from LDS while the MFMAs of
  // step s run
  constexpr int NKS = BK / F::KT;
  static_assert(NKS % 2 == 0, "even number of k-steps per tile");
  T af[2][FM], bf[2][FN];
  auto read_frag = [&](int slot, const T* as, const T* bs, int ks) {
#pragma unroll
    for (int i = 0; i < FM; ++i) af[slot][i] = as[(ks + lane / F::MT) * LDA + wm + i * F::MT + lane % F::MT];
#pragma unroll
    for (int j = 0; j < FN; ++j) bf[slot][j] = bs[(ks + lane / F::NT) * LDB + wn + j * F::NT + lane % F::NT];
  };
  auto mma = [&](int slot) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = F::mma(af[slot][i], bf[slot][j], acc[i][j]);
  };

  // Pipeline per tile t (one barrier): the MFMAs read tile t from LDS buffer t&1; at the start of the tile,
  // tile t+1 (in registers since the start of tile t-1) is staged into the other buffer, whose last reads ended
  // at the previous barrier, and tile t+2 is loaded into registers, a whole tile ahead of its use. The barrier
  // sits before the last k-step, after which the first fragments of tile t+1 are read. FULL: tiles t+1 and t+2
  // exist and t+1 is complete (the steady state, without branches).
  auto tile = [&](auto full_tag, int64_t kt, int buf) {
    constexpr bool FULL = decltype(full_tag)::value;
    const T* as = As[buf];
    const T* bs = Bs[buf];
    if (FULL) {
      // the staging and the global reads stay in the first k-step's scheduling region (the fence keeps the
      // compiler from sinking the reads towards the end of the tile, which would shorten their lead)
      read_frag(1, as, bs, F::KT);
      mma(0);
      la.template store<LDA, false>(As[buf ^ 1], kt + BK, ke);
      lb.template store<LDB, false>(Bs[buf ^ 1], kt + BK, ke);
      la.load(kt + 2 * BK, g.K, g.kl, g.kl.sa);
      lb.load(kt + 2 * BK, g.K, g.kl, g.kl.sb);
      __builtin_amdgcn_sched_barrier(0);
    } else {
      if (kt + BK < ke) {
        la.template store_tile<LDA>(As[buf ^ 1], kt + BK, ke);
        lb.template store_tile<LDB>(Bs[buf ^ 1], kt + BK, ke);
        if (kt + 2 * BK < ke) {
          la.load(kt + 2 * BK, g.K, g.kl, g.kl.sa);
          lb.load(kt + 2 * BK, g.K, g.kl, g.kl.sb);
        }
      }
      read_frag(1, as, bs, F::KT);
      mma(0);
    }
#pragma unroll
    for (int ks = 1; ks + 1 < NKS; ++ks) {
      read_frag((ks + 1) & 1, as, bs, (ks + 1) * F::KT);
      mma(ks & 1);
    }
    __syncthreads();
    if (FULL || kt + BK < ke) read_frag(0, As[buf ^ 1], Bs[buf ^ 1], 0);
    mma((NKS - 1) & 1);
  };

  if (kb < ke) {
    la.load(kb, g.K, g.kl, g.kl.sa);
    lb.load(kb, g.K, g.kl, g.kl.sb);
    la.template store_tile<LDA>(As[0], kb, ke);
    lb.template store_tile<LDB>(Bs[0], kb, ke);
    if (kb + BK < ke) {
      la.load(kb + BK, g.K, g.kl, g.kl.sa);
      lb.load(kb + BK, g.K, g.kl, g.kl.sb);
    }
  }
  __syncthreads();
  if (kb < ke) read_frag(0, As[0], Bs[0], 0);
  int64_t kt = kb;
  int buf = 0;
  for (; kt + 2 * BK < ke; kt += BK, buf ^= 1) tile(std::true_type{}, kt, buf);
  for (; kt < ke; kt += BK, buf ^= 1) tile(std::false_type{}, kt, buf);

  // epilogue
  if (g.split) {
    T* P = static_cast<T*>(g.partial[grp]) + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < F::NACC; ++r) {
          int64_t row = m0 + wm + i * F::MT + F::row(lane, r);
          int64_t col = n0 + wn + j * F::NT + F::col(lane);
          if (row < g.M && col < g.N) P[row * g.N + col] = acc[i][j][r];
        }
    return;
  }
  T* __restrict__ C = static_cast<T*>(g.C[grp]);
  const T alpha = T(g.alpha), beta = T(g.beta);
  // table lookups first (padded: always in range), then the masked stores
  int64_t cn[FN];
  bool cv[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int64_t col = n0 + wn + j * F::NT + F::col(lane);
    cn[j] = g.c_n[col];
    cv[j] = col < g.N;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    int64_t cm[F::NACC];
    bool rv[F::NACC];
#pragma unroll
    for (int r = 0; r < F::NACC; ++r) {
      const int64_t row = m0 + wm + i * F::MT + F::row(lane, r);
      cm[r] = g.c_m[row];
      rv[r] = row < g.M;
    }
    if (g.beta != 0.0) {
      // per MFMA block, all reads of C first, unconditionally (padded table entries address element 0 of a
      // valid row or column), so they are in flight together; then the masked read-modify-write stores
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        T cold[F::NACC];
#pragma unroll
        for (int r = 0; r < F::NACC; ++r) cold[r] = C[cm[r] + cn[j]];
#pragma unroll
        for (int r = 0; r < F::NACC; ++r)
          if (cv[j] && rv[r]) C[cm[r] + cn[j]] = alpha * acc[i][j][r] + beta * cold[r];
      }
    } else {
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < F::NACC; ++r)
          if (cv[j] && rv[r]) C[cm[r] + cn[j]] = alpha * acc[i][j][r];
    }
  }
}

// ---- split-bf16 (hi + lo) form: C ~= A_hi B_hi + A_hi B_lo + A_lo B_hi on the bf16 MFMA ------------------

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// The same split for two elements: one packed conversion gives both hi values, whose FP32 values are the packed
// word's halves moved to the top 16 bits (the subtraction is exact), then one packed conversion of the two lo.
// The empty asm statement (no instruction) hides the packed word's origin from the optimiser, which would
// otherwise convert x0 a second time to rebuild its FP32 hi.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline void split_bf16x2(float x0, float x1, bf16x2& hi, bf16x2& lo) {
  uint32_t hb = __builtin_bit_cast(uint32_t, bf16x2{(__bf16)x0, (__bf16)x1});
  __asm__("" : "+v"(hb));
  hi = __builtin_bit_cast(bf16x2, hb);
  const float h0 = __uint_as_float(hb << 16), h1 = __uint_as_float(hb & 0xffff0000u);
  lo = bf16x2{(__bf16)(x0 - h0), (__bf16)(x1 - h1)};
}

// Epilogue of the split-bf16 kernels: 16 x 16 accumulator blocks (acc[i] -> row 4 (lane / 16) + i, col lane % 16),
// written as split-K partials or as C = alpha acc + beta C through the C offset tables.
template <int FM, int FN>
__device__ inline void bf16x3_epilogue(const Args& g, const f32x4 (&acc)[FM][FN], int64_t m0, int64_t n0, int wm,
                                       int wn, int lane, int grp) {
  if (g.split) {
    float* P = static_cast<float*>(g.partial[grp]) + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
          int64_t col = n0 + wn + j * 16 + (lane & 15);
          if (row < g.M && col < g.N) P[row * g.N + col] = acc[i][j][r];
        }
    return;
  }
  float* __restrict__ C = static_cast<float*>(g.C[grp]);
  const float alpha = float(g.alpha), beta = float(g.beta);
  int64_t cn[FN];
  bool cv[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int64_t col = n0 + wn + j * 16 + (lane & 15);
    cn[j] = g.c_n[col];
    cv[j] = col < g.N;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    int64_t cm[4];
    bool rv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
      cm[r] = g.c_m[row];
      rv[r] = row < g.M;
    }
    float cold[FN][4];
    if (g.beta != 0.0) {
      // unconditional reads first (padded table entries address a valid element), then the masked stores
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) cold[j][r] = C[cm[r] + cn[j]];
    }
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (cv[j] && rv[r]) {
          float v = alpha * acc[i][j][r];
          if (g.beta != 0.0) v += beta * cold[j][r];
          C[cm[r] + cn[j]] = v;
        }
  }
}

// FP32 tiles are split into bf16 hi and lo planes when staged in LDS. Each plane is stored row-major with k
// contiguous (row pitch BK + 8 bf16 = 80 bytes), so a lane's 8-element MFMA fragment is one 16-byte LDS read.
template <int BM, int BN, int BK, bool AKF, bool BKF, int NKL>
__global__ void __launch_bounds__(256) gett_bf16x3_kernel(Args g) {
  static_assert(BK == 32, "one bf16 MFMA step per tile");
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LDK = BK + 8;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Al[BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[BN * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * WM;
  const int wn = (wave & 1) * WN;
  int64_t m0, n0;
  tile_origin<BM, BN>(xcd_tile(blockIdx.x, gridDim.x), g.M, g.N, m0, n0);
  const int64_t kb = (int64_t)blockIdx.z * g.kchunk;
  const int64_t ke = (g.K < kb + g.kchunk) ? g.K : kb + g.kchunk;
  const int grp = blockIdx.y;
  const float* __restrict__ A = static_cast<const float*>(g.A[grp]);
  const float* __restrict__ B = static_cast<const float*>(g.B[grp]);

  Loader<float, BM, BK, AKF, NKL> la;
  Loader<float, BN, BK, BKF, NKL> lb;
  la.init(A, g.a_m, m0, tid);
  lb.init(B, g.b_n, n0, tid);

  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  if (kb < ke) {
    la.load(kb, g.K, g.kl, g.kl.sa);
    lb.load(kb, g.K, g.kl, g.kl.sb);
  }
  const int kq = 8 * (lane >> 4);
  for (int64_t kt = kb; kt < ke; kt += BK) {
#pragma unroll
    for (int i = 0; i < la.PER; ++i) {
      __bf16 h, l;
      split_bf16(la.template value<true>(i, kt, ke), h, l);
      const int r = la.r0 + (i % la.NR) * la.RSTEP, k = la.k0 + (i / la.NR) * la.KSTEP;
      Ah[r * LDK + k] = h;
      Al[r * LDK + k] = l;
    }
#pragma unroll
    for (int i = 0; i < lb.PER; ++i) {
      __bf16 h, l;
      split_bf16(lb.template value<true>(i, kt, ke), h, l);
      const int r = lb.r0 + (i % lb.NR) * lb.RSTEP, k = lb.k0 + (i / lb.NR) * lb.KSTEP;
      Bh[r * LDK + k] = h;
      Bl[r * LDK + k] = l;
    }
    __syncthreads();
    if (kt + BK < ke) {
      la.load(kt + BK, g.K, g.kl, g.kl.sa);
      lb.load(kt + BK, g.K, g.kl, g.kl.sb);
    }
    bf16x8 bh[FN], bl[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int c = (wn + j * 16 + (lane & 15)) * LDK + kq;
      bh[j] = *reinterpret_cast<const bf16x8*>(&Bh[c]);
      bl[j] = *reinterpret_cast<const bf16x8*>(&Bl[c]);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r = (wm + i * 16 + (lane & 15)) * LDK + kq;
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&Ah[r]);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(&Al[r]);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  bf16x3_epilogue<FM, FN>(g, acc, m0, n0, wm, wn, lane, grp);
}

// Split-bf16 form with 16-byte tile loads (both operands' layouts allow them): 128 x 128 tiles, BK = 32, each
// thread loading four 4-element vectors per operand and tile. Thread t owns rows 4 (t / 8) .. 4 (t / 8) + 3 and
// k 4 (t % 8) .. 4 (t % 8) + 3 of the tile. A k-walking operand's vector is 4 consecutive k of one row; a
// row-walking operand's four vectors are the same 4 rows at 4 consecutive k, transposed in registers. Either way a
// thread stages 4 k of a row at a time: split into hi and lo and written as one 8-byte LDS store per plane (planes
// row-major with k contiguous, pitch BK + 8, as in the kernel above). Eight consecutive lanes fill 64 contiguous
// bytes of one row and the next eight lanes start 4 rows (80 dwords) further, so the stores of 32 lanes cover 64
// distinct banks; with the older assignment (a row-walking thread on rows 4 (t % 32) ..) 32 lanes wrote 4 rows
// apart at one k, all into 4 bank pairs, and the kernel spent over a third of its wave cycles waiting on LDS.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
template <bool KFAST, int NKL>
struct Bf16VecLoader {
  static constexpr int BMN = 128, BK = 32, LDK = BK + 8;
  const float* rowp[4];
  int r0, k0;
  f32x4 reg[4];

  __device__ inline void init(const float* base, const int64_t* off_r, int64_t rbase, int tid) {
    r0 = 4 * (tid / 8);  // rows r0 .. r0 + 3
    k0 = 4 * (tid % 8);
    if (KFAST) {
#pragma unroll
      for (int i = 0; i < 4; ++i) rowp[i] = base + off_r[rbase + r0 + i];
    } else {
      rowp[0] = base + off_r[rbase + r0];
    }
  }
  // The fastest contracted leg's extent is a multiple of 4 (required by the launch), and kt + k0 is one too, so
  // the thread's 4 k's differ only in that leg's digit: one offset, then steps of that leg's stride.
  __device__ inline void load(int64_t kt, int64_t K, const GettKLegs& kl, const uint32_t* stride) {
    const uint32_t k = (uint32_t)kt + (uint32_t)k0, klast = (uint32_t)K - 4;
    const uint64_t o = k_offset<NKL>(k < klast ? k : klast, kl, stride);
    if (KFAST) {
#pragma unroll
      for (int i = 0; i < 4; ++i) reg[i] = *reinterpret_cast<const f32x4*>(rowp[i] + o);
    } else {
      const float* p = rowp[0] + o;
      const uint64_t s0 = stride[0];
#pragma unroll
      for (int j = 0; j < 4; ++j) reg[j] = *reinterpret_cast<const f32x4*>(p + j * s0);
    }
  }
  // stages the tile starting at kt; KMASK: zero past kend
  template <bool KMASK>
  __device__ inline void store(__bf16* hi, __bf16* lo, int64_t kt, int64_t kend) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        x[j] = KFAST ? reg[i][j] : reg[j][i];
        if (KMASK && kt + k0 + j >= kend) x[j] = 0.f;
      }
      bf16x2 h01, l01, h23, l23;
      split_bf16x2(x[0], x[1], h01, l01);
      split_bf16x2(x[2], x[3], h23, l23);
      const bf16x4 h{h01[0], h01[1], h23[0], h23[1]}, l{l01[0], l01[1], l23[0], l23[1]};
      const int row = r0 + i;
      *reinterpret_cast<bf16x4*>(&hi[row * LDK + k0]) = h;
      *reinterpret_cast<bf16x4*>(&lo[row * LDK + k0]) = l;
    }
  }
  __device__ inline void store_tile(__bf16* hi, __bf16* lo, int64_t kt, int64_t kend) const {
    if (kt + BK <= kend) store<false>(hi, lo, kt, kend);
    else store<true>(hi, lo, kt, kend);
  }
};

// Pipeline as in gett_kernel: double-buffered planes, tile t+1 staged from registers at the start of tile t and
// tile t+2 loaded right after (fenced), one barrier per tile; one MFMA k-step (k = 32) per tile.
template <bool AKF, bool BKF, int NKL>
__global__ void __launch_bounds__(256, 2) gett_bf16x3_vec_kernel(Args g) {
  constexpr int BM = 128, BN = 128, BK = 32, LDK = BK + 8;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BN * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * WM;
  const int wn = (wave & 1) * WN;
  int64_t m0, n0;
  tile_origin<BM, BN>(xcd_tile(blockIdx.x, gridDim.x), g.M, g.N, m0, n0);
  const int64_t kb = (int64_t)blockIdx.z * g.kchunk;
  const int64_t ke = (g.K < kb + g.kchunk) ? g.K : kb + g.kchunk;
  const int grp = blockIdx.y;
  const float* __restrict__ A = static_cast<const float*>(g.A[grp]);
  const float* __restrict__ B = static_cast<const float*>(g.B[grp]);

  Bf16VecLoader<AKF, NKL> la;
  Bf16VecLoader<BKF, NKL> lb;
  la.init(A, g.a_m, m0, tid);
  lb.init(B, g.b_n, n0, tid);

  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int kq = 8 * (lane >> 4);
  auto compute = [&](int buf) {
    bf16x8 bh[FN], bl[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int c = (wn + j * 16 + (lane & 15)) * LDK + kq;
      bh[j] = *reinterpret_cast<const bf16x8*>(&Bh[buf][c]);
      bl[j] = *reinterpret_cast<const bf16x8*>(&Bl[buf][c]);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r = (wm + i * 16 + (lane & 15)) * LDK + kq;
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&Ah[buf][r]);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(&Al[buf][r]);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
      }
    }
  };

  if (kb < ke) {
    la.load(kb, g.K, g.kl, g.kl.sa);
    lb.load(kb, g.K, g.kl, g.kl.sb);
    la.store_tile(Ah[0], Al[0], kb, ke);
    lb.store_tile(Bh[0], Bl[0], kb, ke);
    if (kb + BK < ke) {
      la.load(kb + BK, g.K, g.kl, g.kl.sa);
      lb.load(kb + BK, g.K, g.kl, g.kl.sb);
    }
  }
  __syncthreads();
  int buf = 0;
  for (int64_t kt = kb; kt < ke; kt += BK, buf ^= 1) {
    if (kt + 2 * BK < ke) {
      la.template store<false>(Ah[buf ^ 1], Al[buf ^ 1], kt + BK, ke);
      lb.template store<false>(Bh[buf ^ 1], Bl[buf ^ 1], kt + BK, ke);
      la.load(kt + 2 * BK, g.K, g.kl, g.kl.sa);
      lb.load(kt + 2 * BK, g.K, g.kl, g.kl.sb);
      __builtin_amdgcn_sched_barrier(0);
    } else if (kt + BK < ke) {
      la.store_tile(Ah[buf ^ 1], Al[buf ^ 1], kt + BK, ke);
      lb.store_tile(Bh[buf ^ 1], Bl[buf ^ 1], kt + BK, ke);
    }
    compute(buf);
    __syncthreads();
  }
  bf16x3_epilogue<FM, FN>(g, acc, m0, n0, wm, wn, lane, grp);
}

struct RedArgs {
  const void* P[kGettMaxGroup];
  void* C[kGettMaxGroup];
};

template <typename T>
__global__ void splitk_reduce_kernel(RedArgs r, int splits, int64_t M, int64_t N, const int64_t* __restrict__ c_m,
                                     const int64_t* __restrict__ c_n, double alpha, double beta) {
  const T* __restrict__ P = static_cast<const T*>(r.P[blockIdx.y]);
  T* C = static_cast<T*>(r.C[blockIdx.y]);
  const int64_t total = M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += (double)P[(int64_t)z * total + idx];
    int64_t m = idx / N, n = idx - m * N;
    int64_t o = c_m[m] + c_n[n];
    double v = alpha * s;
    if (beta != 0.0) v += beta * (double)C[o];
    C[o] = (T)v;
  }
}

template <typename T, int BM, int BN, int BK, int NKL, bool VEC>
void launch_tile_k(const Args& a, dim3 grid, hipStream_t s, bool akf, bool bkf) {
  const dim3 block(256);
  if (akf && bkf) hipLaunchKernelGGL((gett_kernel<T, BM, BN, BK, true, true, NKL, VEC>), grid, block, 0, s, a);
  else if (akf) hipLaunchKernelGGL((gett_kernel<T, BM, BN, BK, true, false, NKL, VEC>), grid, block, 0, s, a);
  else if (bkf) hipLaunchKernelGGL((gett_kernel<T, BM, BN, BK, false, true, NKL, VEC>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gett_kernel<T, BM, BN, BK, false, false, NKL, VEC>), grid, block, 0, s, a);
}

// Kernels are instantiated for 2 and for 4 contracted legs (fewer legs run with zero entries), with scalar or
// vector tile loads.
template <typename T, int BM, int BN, int BK>
void launch_tile(const Args& a, int groups, int splits, hipStream_t s, bool akf, bool bkf, bool vec) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const dim3 grid((unsigned)tiles, (unsigned)groups, (unsigned)splits);
  if (vec) {
    if (a.kl.n <= 2) launch_tile_k<T, BM, BN, BK, 2, true>(a, grid, s, akf, bkf);
    else launch_tile_k<T, BM, BN, BK, 4, true>(a, grid, s, akf, bkf);
  } else {
    if (a.kl.n <= 2) launch_tile_k<T, BM, BN, BK, 2, false>(a, grid, s, akf, bkf);
    else launch_tile_k<T, BM, BN, BK, 4, false>(a, grid, s, akf, bkf);
  }
}

template <int BM, int BN, int BK, int NKL>
void launch_bf16x3_k(const Args& a, dim3 grid, hipStream_t s, bool akf, bool bkf) {
  const dim3 block(256);
  if (akf && bkf) hipLaunchKernelGGL((gett_bf16x3_kernel<BM, BN, BK, true, true, NKL>), grid, block, 0, s, a);
  else if (akf) hipLaunchKernelGGL((gett_bf16x3_kernel<BM, BN, BK, true, false, NKL>), grid, block, 0, s, a);
  else if (bkf) hipLaunchKernelGGL((gett_bf16x3_kernel<BM, BN, BK, false, true, NKL>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gett_bf16x3_kernel<BM, BN, BK, false, false, NKL>), grid, block, 0, s, a);
}

template <int NKL>
void launch_bf16x3_vec_k(const Args& a, dim3 grid, hipStream_t s, bool akf, bool bkf) {
  const dim3 block(256);
  if (akf && bkf) hipLaunchKernelGGL((gett_bf16x3_vec_kernel<true, true, NKL>), grid, block, 0, s, a);
  else if (akf) hipLaunchKernelGGL((gett_bf16x3_vec_kernel<true, false, NKL>), grid, block, 0, s, a);
  else if (bkf) hipLaunchKernelGGL((gett_bf16x3_vec_kernel<false, true, NKL>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gett_bf16x3_vec_kernel<false, false, NKL>), grid, block, 0, s, a);
}

template <int BM, int BN, int BK>
void launch_bf16x3(const Args& a, int groups, int splits, hipStream_t s, bool akf, bool bkf, bool vec) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const dim3 grid((unsigned)tiles, (unsigned)groups, (unsigned)splits);
  if constexpr (BM == 128 && BN == 128 && BK == 32) {
    if (vec) {
      if (a.kl.n <= 2) launch_bf16x3_vec_k<2>(a, grid, s, akf, bkf);
      else launch_bf16x3_vec_k<4>(a, grid, s, akf, bkf);
      return;
    }
  }
  if (a.kl.n <= 2) launch_bf16x3_k<BM, BN, BK, 2>(a, grid, s, akf, bkf);
  else launch_bf16x3_k<BM, BN, BK, 4>(a, grid, s, akf, bkf);
}

struct Tile {
  int bm, bn;
};

// Tile shape per precision and extents. FP64: 128 x 64 (the 128 x 128 FP64 tile gives no gain at its lower
// occupancy). FP32: among 192 x 192, 128 x 192, 192 x 128 and 128 x 128 the one with the least padding, ties to
// the larger tile (higher arithmetic intensity; the 192 x 192 tile runs the chi = 24 steps about 5 % faster);
// chi^2 = 576 and chi^4 extents at chi = 24 are multiples of 192 but not of 128. A 192-row (column) tile is only
// chosen when it pads no more than a 128-row one, so the offset tables, padded to multiples of 128, cover every
// tile. BF16X3: at most 128 x 128. 64-wide tiles for extents below 128.
Tile choose_tile(Prec p, int64_t M, int64_t N) {
  const bool bigm = M >= 128, bign = N >= 128;
  if (p == Prec::F64) return Tile{bigm ? 128 : 64, 64};
  if (p == Prec::BF16X3 || !bigm || !bign) return Tile{bigm ? 128 : 64, bign ? 128 : 64};
  const Tile cand[4] = {{192, 192}, {128, 192}, {192, 128}, {128, 128}};
  Tile best = cand[3];
  double best_pad = 1e300;
  for (const Tile& c : cand) {
    if (M < c.bm || N < c.bn) continue;
    const double pad = (double)((M + c.bm - 1) / c.bm * c.bm) * (double)((N + c.bn - 1) / c.bn * c.bn);
    if (pad < best_pad * (1 - 1e-12)) {
      best = c;
      best_pad = pad;
    }
  }
  return best;
}

}  // namespace

void gett_run(Ctx& ctx, const GettTables& t, const GettLaunch& l) {
  if (t.M <= 0 || t.N <= 0) return;
  const int G = l.groups;
  if (G < 1 || G > kGettMaxGroup) throw Error(MERA_EINVAL, "gett: group count out of range");
  Args a{};
  for (int g = 0; g < G; ++g) {
    a.A[g] = l.A[g];
    a.B[g] = l.B[g];
    a.C[g] = l.C[g];
  }
  a.a_m = t.a_m;
  a.b_n = t.b_n;
  a.kl = t.kl;
  a.c_m = t.c_m;
  a.c_n = t.c_n;
  a.M = t.M;
  a.N = t.N;
  a.K = t.K;
  a.alpha = l.alpha;
  a.beta = l.beta;
  a.split = 0;

  const Tile tile = choose_tile(l.prec, t.M, t.N);
  const int BMsel = tile.bm, BNsel = tile.bn;
  // the m and n offset tables are padded to multiples of 128; every tile must lie within them
  auto rup = [](int64_t x, int64_t m) { return (x + m - 1) / m * m; };
  if (rup(t.M, BMsel) > rup(t.M, 128) || rup(t.N, BNsel) > rup(t.N, 128))
    throw Error(MERA_EINVAL, "gett: tile exceeds the padded offset tables");
  const int64_t tiles = ((t.M + BMsel - 1) / BMsel) * ((t.N + BNsel - 1) / BNsel);
  const int BK = 32;  // k-chunks stay multiples of every tile depth in use

  // split-K when the output grid cannot fill the chip and K is long
  int splits = l.splits;
  if (splits <= 0) {
    splits = 1;
    const int64_t target = 1024;
    while (tiles * splits < target && t.K / (splits * 2) >= 512 && splits < 64) splits *= 2;
  }
  int64_t kchunk = (t.K + splits - 1) / splits;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  splits = (int)std::max<int64_t>(1, (t.K + kchunk - 1) / kchunk);
  a.kchunk = kchunk;

  const size_t eb = (l.prec == Prec::F64) ? 8 : 4;
  if (splits > 1) {
    const size_t per = (size_t)splits * t.M * t.N * eb;
    char* p = static_cast<char*>(ctx.buf("gett.partial", per * G));
    for (int g = 0; g < G; ++g) a.partial[g] = p + per * g;
    a.split = 1;
  }
  if (l.prepare_only) return;
  // vector tile loads when both operands' layouts allow them (planned) and every base is 16-byte aligned
  const int vw = l.prec == Prec::F64 ? 2 : 4;
  bool vec = t.a_vw >= vw && t.b_vw >= vw;
  for (int g = 0; g < G; ++g)
    vec = vec && ((uintptr_t)l.A[g] % 16 == 0) && ((uintptr_t)l.B[g] % 16 == 0);
  // the vector split-bf16 kernel's tile; its loads take 4 consecutive k within the fastest contracted leg
  if (l.prec == Prec::BF16X3) vec = vec && BMsel == 128 && BNsel == 128 && t.kl.n >= 1 && t.kl.ext[0] % 4 == 0;
  hipStream_t s = ctx.stream;
  LaunchRecord rec;
  if (ctx.profiling) {
    rec.kernel = std::string("gett<") + (l.prec == Prec::F64 ? "f64" : (l.prec == Prec::F32 ? "f32" : "bf16x3")) +
                 "," + std::to_string(BMsel) + "x" + std::to_string(BNsel) + (t.a_kfast ? ",Ak" : ",Am") +
                 (t.b_kfast ? ",Bk" : ",Bn") + (vec ? ",v" : "") + (t.kl.n <= 2 ? ",k2" : ",k4") +
                 (splits > 1 ? ",splitk" : "") + (G > 1 ? ",grouped" : "") + ">";
    rec.flops = 2.0 * G * (double)t.M * (double)t.N * (double)t.K;
    rec.bytes = G * (double)eb * ((double)t.M * t.K + (double)t.K * t.N + (double)t.M * t.N * (l.beta != 0.0 ? 2 : 1));
    rec.start = ctx.take_event();
    rec.stop = ctx.take_event();
    MERA_HIP(hipEventRecord(rec.start, s));
  }
  const int sel = BMsel * 1000 + BNsel;
  const bool akf = t.a_kfast, bkf = t.b_kfast;

  if (l.prec == Prec::F64) {
    if (sel == 128064) launch_tile<double, 128, 64, 16>(a, G, splits, s, akf, bkf, vec);
    else launch_tile<double, 64, 64, 16>(a, G, splits, s, akf, bkf, vec);
  } else if (l.prec == Prec::F32) {
    switch (sel) {
      case 192192: launch_tile<float, 192, 192, 16>(a, G, splits, s, akf, bkf, vec); break;
      case 128192: launch_tile<float, 128, 192, 16>(a, G, splits, s, akf, bkf, vec); break;
      case 192128: launch_tile<float, 192, 128, 16>(a, G, splits, s, akf, bkf, vec); break;
      case 128128: launch_tile<float, 128, 128, 16>(a, G, splits, s, akf, bkf, vec); break;
      case 128064: launch_tile<float, 128, 64, 16>(a, G, splits, s, akf, bkf, vec); break;
      case 64128: launch_tile<float, 64, 128, 16>(a, G, splits, s, akf, bkf, vec); break;
      default: launch_tile<float, 64, 64, 16>(a, G, splits, s, akf, bkf, vec); break;
    }
  } else {
    switch (sel) {
      case 128128: launch_bf16x3<128, 128, 32>(a, G, splits, s, akf, bkf, vec); break;
      case 128064: launch_bf16x3<128, 64, 32>(a, G, splits, s, akf, bkf, vec); break;
      case 64128: launch_bf16x3<64, 128, 32>(a, G, splits, s, akf, bkf, vec); break;
      default: launch_bf16x3<64, 64, 32>(a, G, splits, s, akf, bkf, vec); break;
    }
  }
  MERA_HIP(hipGetLastError());
  if (ctx.profiling) {
    MERA_HIP(hipEventRecord(rec.stop, s));
    ctx.records.push_back(rec);
  }
  if (splits > 1) {
    RedArgs r{};
    for (int g = 0; g < G; ++g) {
      r.P[g] = a.partial[g];
      r.C[g] = l.C[g];
    }
    const int64_t total = t.M * t.N;
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    if (l.prec == Prec::F64)
      hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3(blocks, G), dim3(256), 0, s, r, splits, t.M, t.N, t.c_m,
                         t.c_n, l.alpha, l.beta);
    else
      hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3(blocks, G), dim3(256), 0, s, r, splits, t.M, t.N, t.c_m,
                         t.c_n, l.alpha, l.beta);
    MERA_HIP(hipGetLastError());
  }
}

}  // namespace mera
