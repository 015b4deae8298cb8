// HIP kernels of the GMRF posterior path for gfx950 (MI355X).
//
// Numeric phase = multifrontal supernodal Cholesky of P Q^ P^T (Sec. 3.2), scheduled by
// depth of the supernodal elimination tree: every front of one depth is processed by
// the same batched launch.  Dense front work is blocked in 64-wide column blocks:
//   * diagonal 64x64 blocks are factored in FP64 in LDS (also in the FP32 mode) and
//     inverted (the inverse drives the panel TRSM and the solves),
//   * panel TRSM and the inner panel update are 64x64 MFMA tiles, the long-K products
//     (outer panel update, trailing SYRK, Sigma[R', K]) 128x128 FP64 tiles or, in the
//     FP32 mode, 256x256 tiles whose FP32 products run as six bf16 MFMA term products
//     (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32 / v_mfma_f32_32x32x16_bf16),
//     operands staged in LDS,
//   * children's update matrices are pulled into the parent front one child slot at
//     a time (deterministic, no floating-point atomics).
// Solves pass update vectors up the tree (forward) and read ancestors' solution
// entries (backward).  Selected inversion runs the blocked Takahashi recursion on a
// square Sigma front per supernode, top-down (Sec. 3.2, marginal variances).
#include "kernels.h"

#include <climits>
#include <type_traits>

namespace gmrf {

namespace {

constexpr int kThreads = 256;
constexpr int kP = 80;        // LDS row pitch of the MFMA operand tiles (bank spread)
constexpr int kTK = 16;       // K chunk of the MFMA tile loop
constexpr int kSub = kNB2 / kNB;
constexpr int kExtUnroll = 4;  // relative-index batches in flight per thread

template <typename T> struct V4;
template <> struct V4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <> struct V4<float> { typedef float type __attribute__((ext_vector_type(4))); };

__device__ __forceinline__ V4<double>::type mfma(double a, double b, V4<double>::type c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ V4<float>::type mfma(float a, float b, V4<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int fn(const DevSym& S, int s) { return (int)(S.rowptr[s + 1] - S.rowptr[s]); }
__device__ __forceinline__ int fp(const DevSym& S, int s) { return S.sfirst[s + 1] - S.sfirst[s]; }

// work-group -> (list index, local work-group index): one load from the list's
// work-group map; lists without a map (a single front, or a map too large to keep)
// fall back to a binary search on the prefix
__device__ __forceinline__ void find_front(const LaunchList& L, int64_t wg, int& fi, int64_t& loc) {
  if (L.count == 1) {
    fi = 0;
    loc = wg;
    return;
  }
  if (L.wgmap) {
    const int2 m = L.wgmap[wg];
    fi = m.x;
    loc = m.y;
    return;
  }
  int lo = 0, hi = L.count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (L.prefix[mid] <= wg) lo = mid; else hi = mid - 1;
  }
  fi = lo;
  loc = wg - L.prefix[lo];
}

__device__ __forceinline__ int64_t wg_id() { return (int64_t)blockIdx.x; }

// C(64x64 tile) = sum_k Aop[m][k] Bop[k][n], k < K, rows m < M, cols n < N valid.
//  A_KC=false: Aop[m][k] = A[m + k*lda];  A_KC=true: Aop[m][k] = A[k + m*lda]
//  B_KC=true:  Bop[k][n] = B[k + n*ldb];  B_KC=false: Bop[k][n] = B[n + k*ldb]
// Wave w owns the 32x32 sub-tile at rows 32*(w&1), cols 32*(w>>1): 2x2 MFMA 16x16 blocks.
// acc[i][j][r] holds C[32*(w&1) + 16 i + acc_row<T>(lane, r)][32*(w>>1) + 16 j + (lane&15)].
// sA, sB hold two K chunks each (kTile64Lds elements): the next chunk is loaded into
// registers while the current one is multiplied.  Ends with a barrier, so the buffers
// can be reused by the caller.
constexpr int kTile64Lds = 2 * kTK * kP;

// Loads of one K chunk from clamped addresses (M, N, K >= 1), left unmasked so that no
// consumer sits between them and the multiplication of the current chunk; tile64_store
// zeroes the out-of-range entries.
template <typename T, bool A_KC, bool B_KC>
__device__ __forceinline__ void tile64_load(const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                                            int64_t ldb, int M, int N, int K, int k0, T (&ra)[4], T (&rb)[4]) {
  const int t = threadIdx.x;
  if (!A_KC) {
    const T* Am = A + min(t & 63, M - 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[i] = Am[(int64_t)min(k0 + (t >> 6) + 4 * i, K - 1) * lda];
  } else {
    const T* Ak = A + min(k0 + (t & 15), K - 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[i] = Ak[(int64_t)min((t >> 4) + 16 * i, M - 1) * lda];
  }
  if (!B_KC) {
    const T* Bn = B + min(t & 63, N - 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) rb[i] = Bn[(int64_t)min(k0 + (t >> 6) + 4 * i, K - 1) * ldb];
  } else {
    const T* Bk = B + min(k0 + (t & 15), K - 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) rb[i] = Bk[(int64_t)min((t >> 4) + 16 * i, N - 1) * ldb];
  }
}

template <typename T, bool A_KC, bool B_KC>
__device__ __forceinline__ void tile64_store(T* sA, T* sB, const T (&ra)[4], const T (&rb)[4], int M, int N, int K,
                                             int k0) {
  const int t = threadIdx.x;
  if (!A_KC) {
    const T mm = (T)((t & 63) < M);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = (t >> 6) + 4 * i;
      sA[k * kP + (t & 63)] = ra[i] * (mm * (T)(k0 + k < K));
    }
  } else {
    const T mk = (T)(k0 + (t & 15) < K);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = (t >> 4) + 16 * i;
      sA[(t & 15) * kP + m] = ra[i] * (mk * (T)(m < M));
    }
  }
  if (!B_KC) {
    const T mn = (T)((t & 63) < N);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = (t >> 6) + 4 * i;
      sB[k * kP + (t & 63)] = rb[i] * (mn * (T)(k0 + k < K));
    }
  } else {
    const T mk = (T)(k0 + (t & 15) < K);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int nn = (t >> 4) + 16 * i;
      sB[(t & 15) * kP + nn] = rb[i] * (mk * (T)(nn < N));
    }
  }
}

template <typename T, bool A_KC, bool B_KC>
__device__ __forceinline__ void gemm_tile(const T* __restrict__ A, int64_t lda,
                                          const T* __restrict__ B, int64_t ldb, int M, int N,
                                          int K, typename V4<T>::type (&acc)[2][2], T* sA, T* sB) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  if (K <= 0) return;
  T ra[4], rb[4];
  tile64_load<T, A_KC, B_KC>(A, lda, B, ldb, M, N, K, 0, ra, rb);
  tile64_store<T, A_KC, B_KC>(sA, sB, ra, rb, M, N, K, 0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += kTK) {
    const bool more = k0 + kTK < K;
    if (more) tile64_load<T, A_KC, B_KC>(A, lda, B, ldb, M, N, K, k0 + kTK, ra, rb);
    const T* cA = sA + buf * (kTK * kP);
    const T* cB = sB + buf * (kTK * kP);
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 4) {
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = cA[(kk + (lane >> 4)) * kP + wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = cB[(kk + (lane >> 4)) * kP + wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
    }
    if (more) tile64_store<T, A_KC, B_KC>(sA + (buf ^ 1) * (kTK * kP), sB + (buf ^ 1) * (kTK * kP), ra, rb, M, N, K,
                                            k0 + kTK);
    __syncthreads();
    buf ^= 1;
  }
}

// Loads whose predicate differs per element compile to one branch and one wait per load;
// the kernels below therefore load from clamped (always valid, finite) addresses and mask
// the value afterwards (by a product where the compiler would otherwise sink the load
// into a branch) or predicate only the stores, so that a batch of loads is in flight.

template <typename T>
__device__ __forceinline__ void zero_acc(typename V4<T>::type (&acc)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = typename V4<T>::type{T(0), T(0), T(0), T(0)};
}

// Row of accumulator register r held by `lane` in a 16x16 MFMA output block: the FP32
// 16x16x4 instruction gives each lane 4 consecutive rows, the FP64 one gives rows
// interleaved by 4 (one 64-bit register pair per row group).
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }

// visit every accumulator element with its tile-local (row, col)
template <typename T, typename F>
__device__ __forceinline__ void for_acc(typename V4<T>::type (&acc)[2][2], F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        f(wm + 16 * i + acc_row<T>(lane, r), wn + 16 * j + (lane & 15), acc[i][j][r]);
}

template <typename T, typename F>
__device__ __forceinline__ void for_acc128(typename V4<T>::type (&acc)[4][4], F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        f(wm + 16 * i + acc_row<T>(lane, r), wn + 16 * j + (lane & 15), acc[i][j][r]);
}

// F[gi + gj ld] -= C for the elements of a 64 x 64 (NT = 2) or 128 x 128 (NT = 4) tile
// with r < M, c < N and gi >= gj, gi = row0 + r, gj = col0 + c: all old values are
// loaded first from clamped addresses (M, N >= 1), then the valid ones are stored.
template <typename T, int NT>
__device__ __forceinline__ void acc_sub_lower(const typename V4<T>::type (&acc)[NT][NT], T* F, int64_t ld, int row0,
                                              int col0, int M, int N) {
  constexpr int WS = NT * 16;    // wave sub-tile edge
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * WS, wn = (w >> 1) * WS;
  T old[NT][NT][4];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = min(wm + 16 * i + acc_row<T>(lane, r), M - 1), cc = min(wn + 16 * j + (lane & 15), N - 1);
        old[i][j][r] = F[(row0 + rr) + (int64_t)(col0 + cc) * ld];
      }
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = wm + 16 * i + acc_row<T>(lane, r), cc = wn + 16 * j + (lane & 15);
        const int gi = row0 + rr, gj = col0 + cc;
        if (rr < M && cc < N && gi >= gj) F[gi + (int64_t)gj * ld] = old[i][j][r] - acc[i][j][r];
      }
}


// C(128x128 tile) = sum_k Aop[m][k] Bop[k][n] with the operand conventions of gemm_tile.
// Each wave owns a 64x64 sub-tile (4x4 MFMA 16x16 blocks).  The K loop is software
// pipelined: the next 16-wide K chunk is loaded into registers while the current one,
// double-buffered in LDS, feeds the MFMAs.
constexpr int kBT = 128;
constexpr int kBP = 144;   // LDS pitch: rows of a K slice start 32 banks apart (FP64) / 16 (FP32)

// K chunk of the 128x128 tile (16: the LDS footprint leaves room for several work-groups
// per CU; 32 halved the occupancy and ran slower)
template <typename T> struct BigTK { static constexpr int v = 16; };

// one element of T from a buffer resource: lane byte offset v, scalar byte offset s
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int v, int s) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
}

// Whole chunk (every k of it below K) of two rows-contiguous operands: buffer loads from a
// per-chunk base with the row as the lane offset and the column steps as scalar offsets,
// the same elements big_load reads.  M, N >= 1: every caller's tile holds at least one row
// and one column, so the clamped row offsets are never negative.
template <typename T>
__device__ __forceinline__ void big_load_full(const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                                              int64_t ldb, int M, int N, int k0, T (&ra)[BigTK<T>::v / 2],
                                              T (&rb)[BigTK<T>::v / 2]) {
  constexpr int NL = BigTK<T>::v / 2;
  const int t = threadIdx.x;
  const int kb = k0 + __builtin_amdgcn_readfirstlane(t >> 7);
  const __amdgpu_buffer_rsrc_t sa =
      __builtin_amdgcn_make_buffer_rsrc((void*)(A + (int64_t)kb * lda), (short)0, -1, 0x00020000);
  const __amdgpu_buffer_rsrc_t sb =
      __builtin_amdgcn_make_buffer_rsrc((void*)(B + (int64_t)kb * ldb), (short)0, -1, 0x00020000);
  const int sla = __builtin_amdgcn_readfirstlane((int)(2 * sizeof(T) * lda));
  const int slb = __builtin_amdgcn_readfirstlane((int)(2 * sizeof(T) * ldb));
  const int va = (int)sizeof(T) * min(t & 127, M - 1), vb = (int)sizeof(T) * min(t & 127, N - 1);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    ra[i] = buf_load<T>(sa, va, i * sla);
    rb[i] = buf_load<T>(sb, vb, i * slb);
  }
}

// Same division of work as tile64_load / tile64_store for the 128 x 128 tiles.
template <typename T, bool A_KC, bool B_KC>
__device__ __forceinline__ void big_load(const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                                         int64_t ldb, int M, int N, int K, int k0,
                                         T (&ra)[BigTK<T>::v / 2], T (&rb)[BigTK<T>::v / 2]) {
  constexpr int TK = BigTK<T>::v, NL = TK / 2;
  const int t = threadIdx.x;
  if (!A_KC) {
    const T* Am = A + min(t & 127, M - 1);
#pragma unroll
    for (int i = 0; i < NL; ++i) ra[i] = Am[(int64_t)min(k0 + (t >> 7) + 2 * i, K - 1) * lda];
  } else {
    const T* Ak = A + min(k0 + (t & (TK - 1)), K - 1);
#pragma unroll
    for (int i = 0; i < NL; ++i) ra[i] = Ak[(int64_t)min(t / TK + (kThreads / TK) * i, M - 1) * lda];
  }
  if (!B_KC) {
    const T* Bn = B + min(t & 127, N - 1);
#pragma unroll
    for (int i = 0; i < NL; ++i) rb[i] = Bn[(int64_t)min(k0 + (t >> 7) + 2 * i, K - 1) * ldb];
  } else {
    const T* Bk = B + min(k0 + (t & (TK - 1)), K - 1);
#pragma unroll
    for (int i = 0; i < NL; ++i) rb[i] = Bk[(int64_t)min(t / TK + (kThreads / TK) * i, N - 1) * ldb];
  }
}

template <typename T, bool A_KC, bool B_KC>
__device__ __forceinline__ void big_store(T* sA, T* sB, const T (&ra)[BigTK<T>::v / 2],
                                          const T (&rb)[BigTK<T>::v / 2], int M, int N, int K, int k0) {
  constexpr int TK = BigTK<T>::v, NL = TK / 2;
  const int t = threadIdx.x;
  if (!A_KC) {
    const int m = t & 127;
    const T mm = (T)(m < M);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int k = (t >> 7) + 2 * i;
      sA[k * kBP + m] = ra[i] * (mm * (T)(k0 + k < K));
    }
  } else {
    const int k = t & (TK - 1);
    const T mk = (T)(k0 + k < K);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int m = t / TK + (kThreads / TK) * i;
      sA[k * kBP + m] = ra[i] * (mk * (T)(m < M));
    }
  }
  if (!B_KC) {
    const int nn = t & 127;
    const T mn = (T)(nn < N);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int k = (t >> 7) + 2 * i;
      sB[k * kBP + nn] = rb[i] * (mn * (T)(k0 + k < K));
    }
  } else {
    const int k = t & (TK - 1);
    const T mk = (T)(k0 + k < K);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int nn = t / TK + (kThreads / TK) * i;
      sB[k * kBP + nn] = rb[i] * (mk * (T)(nn < N));
    }
  }
}

// LDS elements per operand (two K-chunk buffers)
template <typename T> struct BigLds { static constexpr int v = 2 * BigTK<T>::v * kBP; };

// sA, sB: BigLds<T>::v elements each
template <typename T, bool A_KC, bool B_KC>
__device__ __forceinline__ void gemm_tile128(const T* __restrict__ A, int64_t lda,
                                             const T* __restrict__ B, int64_t ldb, int M, int N, int K,
                                             typename V4<T>::type (&acc)[4][4], T* sA, T* sB) {
  constexpr int TK = BigTK<T>::v;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
  T ra[TK / 2], rb[TK / 2];
  if (K <= 0) return;
  big_load<T, A_KC, B_KC>(A, lda, B, ldb, M, N, K, 0, ra, rb);
  big_store<T, A_KC, B_KC>(sA, sB, ra, rb, M, N, K, 0);
  __syncthreads();
  int buf = 0;
  // one chunk: fetch chunk k0 + TK, MFMAs of chunk k0 from LDS, store chunk k0 + TK into the
  // idle buffer.  FULL: chunk k0 + TK lies wholly below K and both operands are
  // rows-contiguous, so it is fetched by big_load_full in a loop of its own.
  auto chunk = [&](int k0, auto full) {
    const bool more = k0 + TK < K;
    if constexpr (decltype(full)::value) big_load_full<T>(A, lda, B, ldb, M, N, k0 + TK, ra, rb);
    else if (more) big_load<T, A_KC, B_KC>(A, lda, B, ldb, M, N, K, k0 + TK, ra, rb);
    const T* cA = sA + buf * (TK * kBP);
    const T* cB = sB + buf * (TK * kBP);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = cA[(kk + (lane >> 4)) * kBP + wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = cB[(kk + (lane >> 4)) * kBP + wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
    }
    if (more) big_store<T, A_KC, B_KC>(sA + (buf ^ 1) * (TK * kBP), sB + (buf ^ 1) * (TK * kBP), ra, rb, M, N, K,
                                         k0 + TK);
    __syncthreads();
    buf ^= 1;
  };
  int k0 = 0;
  if constexpr (!A_KC && !B_KC) {
    const int kfull = (K / TK - 1) * TK;   // chunks whose next chunk k0 + TK lies wholly below K
    for (; k0 < kfull; k0 += TK) chunk(k0, std::true_type{});
  }
  for (; k0 < K; k0 += TK) chunk(k0, std::false_type{});
}

template <typename T>
__device__ __forceinline__ void zero_acc128(typename V4<T>::type (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = typename V4<T>::type{T(0), T(0), T(0), T(0)};
}

// ---- FP32 256 x 256 tiles for the long-K products (Sigma[R', K], the left-looking panel
// update, the trailing SYRK) ----
// FP32 products on the bf16 matrix cores.  Each FP32 operand value x is split into three
// bf16 terms x = h + m + l, each the round-to-nearest of what the earlier terms leave, so
// that the residue is below 2^-24 |x|.  A product a b is accumulated in FP32 as the six
// term products of relative order 2^-16 or more (m m, l h, h l, m h, h m, h h, smallest
// first); the three dropped ones are below 2^-24 |a b|.  The result carries the error of
// an FP32 dot product (measured against FP64 dot products it is no larger than that of
// the FP32 16x16x4 MFMA).  For a 32 x 32 x 16 block this takes six 32x32x16 bf16 MFMAs
// instead of sixteen 16x16x4 FP32 ones of the same pass count: 8/3 fewer matrix-core
// cycles.
// Eight waves (2 x 4) with 128 x 64 wave tiles of 4 x 2 blocks of 32 x 32.  Operands are
// staged in 16-wide K chunks, row-major in LDS: a row holds the h, m and l planes of its
// 16 k values (32 bytes each) plus 16 bytes of padding, so a lane's eight k values of one
// plane are one 128-bit read and the 64 lanes of a read fall in distinct bank groups.
// Thread t converts row t & 255, k values 8 (t >> 8) .. +7 of both operands (the
// transpose of the column-major operands happens in registers); the chunks wholly below K
// run in a loop of their own with buffer loads, so that each of its iterations is one
// block of loads, split, LDS traffic and MFMAs for the scheduler to interleave.  Two LDS buffers; the
// registers run one chunk ahead, so that the split of chunk c + 1 into the idle buffer
// and the loads of chunk c + 2 overlap the MFMAs of chunk c.  One work-group covers a
// whole 256-wide outer block, so every row panel is read once per K part.
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f16v_t __attribute__((ext_vector_type(16)));
constexpr int kG4K = 16;   // K chunk
constexpr int kG4 = 256, kThreads4 = 512;
constexpr int kRec4 = 7;   // 16-byte units per LDS row: 3 planes x 2 k halves + padding

__device__ __forceinline__ void zero_acc6(f16v_t (&acc)[4][2]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
}

struct G4Lds {
  uint4 a[2][kG4 * kRec4];
  uint4 b[2][kG4 * kRec4];
};
union __attribute__((aligned(16))) G4Smem {
  G4Lds g;
  float ep[64][kG4 + 1];   // epilogue staging of one 64-column group
};

typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
// round-to-nearest bf16 of (a, b) as one packed pair, and the two values back as floats
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v_t){a, b}, bf2_t));
}
__device__ __forceinline__ float bf16_lo(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

// split of eight values two at a time: each level converts a pair once and subtracts the
// pair's two rounded values from what the earlier levels left
__device__ __forceinline__ void split3_bf16(const float (&x)[8], uint4& h, uint4& m, uint4& l) {
  uint32_t vh[4], vm[4], vl[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t a = pk_bf16(x[2 * q], x[2 * q + 1]);
    const float r0 = x[2 * q] - bf16_lo(a), r1 = x[2 * q + 1] - bf16_hi(a);
    const uint32_t b = pk_bf16(r0, r1);
    vh[q] = a;
    vm[q] = b;
    vl[q] = pk_bf16(r0 - bf16_lo(b), r1 - bf16_hi(b));
  }
  h = make_uint4(vh[0], vh[1], vh[2], vh[3]);
  m = make_uint4(vm[0], vm[1], vm[2], vm[3]);
  l = make_uint4(vl[0], vl[1], vl[2], vl[3]);
}

// row t & 255 (clamped to M - 1, N - 1: the products of such rows land in output rows /
// columns the epilogues discard), k = k0 + 8 (t >> 8) .. +7; values at k >= K are zero.
// FULL: the caller knows that every k of the chunk is below K; the loads are then buffer
// loads from a per-chunk base, with the row as the lane offset and q lda as scalar offsets
// (no address arithmetic per load).  Otherwise the loads come from clamped addresses.
template <bool FULL>
__device__ __forceinline__ void g4_load(const float* __restrict__ A, int64_t lda, const float* __restrict__ B,
                                        int64_t ldb, int M, int N, int K, int k0, float (&ra)[8], float (&rb)[8]) {
  const int t = threadIdx.x;
  const int ra_row = min(t & 255, M - 1), rb_row = min(t & 255, N - 1);
  const int kb = k0 + 8 * __builtin_amdgcn_readfirstlane(t >> 8);
  if constexpr (FULL) {
    const __amdgpu_buffer_rsrc_t sa =
        __builtin_amdgcn_make_buffer_rsrc((void*)(A + (int64_t)kb * lda), (short)0, -1, 0x00020000);
    const __amdgpu_buffer_rsrc_t sb =
        __builtin_amdgcn_make_buffer_rsrc((void*)(B + (int64_t)kb * ldb), (short)0, -1, 0x00020000);
    const int sla = __builtin_amdgcn_readfirstlane((int)(4 * lda)), slb = __builtin_amdgcn_readfirstlane((int)(4 * ldb));
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      ra[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sa, 4 * ra_row, q * sla, 0));
      rb[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sb, 4 * rb_row, q * slb, 0));
    }
  } else {
    const float* Am = A + ra_row;
    const float* Bn = B + rb_row;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t k = min(kb + q, K - 1);
      const bool ok = kb + q < K;
      const float va = Am[k * lda], vb = Bn[k * ldb];
      ra[q] = ok ? va : 0.f;
      rb[q] = ok ? vb : 0.f;
    }
  }
}
// split, store into LDS buffer (a, b)
__device__ __forceinline__ void g4_store(uint4* a, uint4* b, float (&ra)[8], float (&rb)[8]) {
  const int t = threadIdx.x;
  const int u = (t & 255) * kRec4 + (t >> 8);
  uint4 h, m, l;
  split3_bf16(ra, h, m, l);
  a[u] = h; a[u + 2] = m; a[u + 4] = l;
  split3_bf16(rb, h, m, l);
  b[u] = h; b[u + 2] = m; b[u + 4] = l;
}

__device__ __forceinline__ f16v_t mfma_bf16(uint4 a, uint4 b, f16v_t c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8_t, a), __builtin_bit_cast(bf8_t, b), c,
                                                0, 0, 0);
}

// acc += A(M x K) B(N x K)^T for a 256 x 256 tile, both operands column-major.  Rows and
// columns of the result at or beyond M, N are undefined.  Lane l of a wave holds, for
// block (i, j), rows wm + 32 i + 8 (r >> 2) + 4 (l >> 5) + (r & 3) of column
// wn + 32 j + (l & 31) in acc[i][j][r].
__device__ __forceinline__ void gemm_tile4(const float* __restrict__ A, int64_t lda, const float* __restrict__ B,
                                           int64_t ldb, int M, int N, int K, f16v_t (&acc)[4][2], G4Lds& S) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 128, wn = (w >> 1) * 64;
  const int rl = lane & 31, kh = lane >> 5;
  float ra[8], rb[8];
  if (K <= 0) return;
  g4_load<false>(A, lda, B, ldb, M, N, K, 0, ra, rb);
  g4_store(S.a[0], S.b[0], ra, rb);
  g4_load<false>(A, lda, B, ldb, M, N, K, kG4K, ra, rb);
  __syncthreads();
  int buf = 0;
  // one chunk: fragments of chunk k0 from LDS, chunk k0 + 16 (all zero beyond K) split into
  // the idle buffer, chunk k0 + 32 fetched, then the MFMAs of chunk k0
  auto chunk = [&](int k0, auto full) {
    const uint4* cA = S.a[buf];
    const uint4* cB = S.b[buf];
    uint4 bf[2][3], af[4][3];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int p = 0; p < 3; ++p) bf[j][p] = cB[(wn + 32 * j + rl) * kRec4 + 2 * p + kh];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int p = 0; p < 3; ++p) af[i][p] = cA[(wm + 32 * i + rl) * kRec4 + 2 * p + kh];
    g4_store(S.a[buf ^ 1], S.b[buf ^ 1], ra, rb);
    g4_load<decltype(full)::value>(A, lda, B, ldb, M, N, K, k0 + 2 * kG4K, ra, rb);
    constexpr int PA[6] = {1, 2, 0, 1, 0, 0}, PB[6] = {1, 0, 2, 0, 1, 0};
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(af[i][PA[q]], bf[j][PB[q]], acc[i][j]);
    __syncthreads();
    buf ^= 1;
  };
  // the chunks whose prefetched chunk k0 + 32 lies wholly below K, then the rest
  const int kfull = (K / kG4K - 2) * kG4K;
  int k0 = 0;
  for (; k0 < kfull; k0 += kG4K) chunk(k0, std::true_type{});
  for (; k0 < K; k0 += kG4K) chunk(k0, std::false_type{});
}

// columns 64 h .. 64 h + 63 of the tile into sm.ep[column - 64 h][row] (waves w >> 1 == h)
__device__ __forceinline__ void g4_stage(const f16v_t (&acc)[4][2], G4Smem& sm, int h) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if ((w >> 1) != h) return;
  const int wm = (w & 1) * 128;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        sm.ep[32 * j + (lane & 31)][wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)] = acc[i][j][r];
}

// Epilogue of a 256 x 256 tile through LDS, one 64-column group at a time: frow(r, c, v)
// is called with rows fastest across the work-group, then (if COLS) fcol(r, c, v) with
// columns fastest, so that both a column-major block and its transpose are written with
// coalesced accesses.  Starts and ends with a barrier (the staging area aliases the
// operand buffers).
template <bool COLS, typename FR, typename FC>
__device__ __forceinline__ void g4_epilogue(const f16v_t (&acc)[4][2], G4Smem& sm, FR frow, FC fcol) {
  const int t = threadIdx.x;
  for (int h = 0; h < 4; ++h) {
    __syncthreads();
    g4_stage(acc, sm, h);
    __syncthreads();
    for (int e = t; e < kG4 * 64; e += kThreads4) {
      const int row = e & (kG4 - 1), cl = e >> 8;
      frow(row, 64 * h + cl, sm.ep[cl][row]);
    }
    if constexpr (COLS) {
      for (int e = t; e < kG4 * 64; e += kThreads4) {
        const int cl = e & 63, row = e >> 6;
        fcol(row, 64 * h + cl, sm.ep[cl][row]);
      }
    }
  }
  __syncthreads();
}

// F[gi + gj ld] -= C for a 256 x 256 tile (gi = row0 + r, gj = col0 + c, r < M, c < N,
// gi >= gj), staged through LDS one 64-column group at a time; each thread loads the old
// values of a group in batches of 8 from clamped addresses before storing.
__device__ __forceinline__ void g4_epilogue_sub(const f16v_t (&acc)[4][2], G4Smem& sm, float* F, int64_t ld,
                                                int row0, int col0, int M, int N) {
  const int t = threadIdx.x;
  for (int h = 0; h < 4; ++h) {
    __syncthreads();
    g4_stage(acc, sm, h);
    __syncthreads();
    if (64 * h >= N) continue;
#pragma unroll
    for (int e0 = 0; e0 < kG4 * 64; e0 += 8 * kThreads4) {
      float old[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads4 + t;
        const int row = min(e & (kG4 - 1), M - 1), c = min(64 * h + (e >> 8), N - 1);
        old[u] = F[(row0 + row) + (int64_t)(col0 + c) * ld];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads4 + t;
        const int row = e & (kG4 - 1), cl = e >> 8, c = 64 * h + cl;
        const int gi = row0 + row, gj = col0 + c;
        if (row < M && c < N && gi >= gj) F[gi + (int64_t)gj * ld] = old[u] - sm.ep[cl][row];
      }
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ assembly kernels
__global__ void k_assemble_qpost(int64_t nnzq, const double* __restrict__ qval,
                                 const int64_t* __restrict__ cptr, const int32_t* __restrict__ cpair,
                                 const int32_t* __restrict__ arow, const double* __restrict__ aval,
                                 const double* __restrict__ qeps, double* __restrict__ qpost) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnzq;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = qval[e];
    for (int64_t c = cptr[e]; c < cptr[e + 1]; ++c) {
      const int32_t a1 = cpair[2 * c], a2 = cpair[2 * c + 1];
      v += qeps[arow[a1]] * aval[a1] * aval[a2];
    }
    qpost[e] = v;
  }
}

// Derivative of the conditioning on Q's pattern (Sec. 3.1): for a parameter theta,
//   dQ_post = dQ + dA^T Q_eps A + A^T Q_eps dA + A^T diag(dq_eps) A,
// over the same per-entry pairs of A entries that assemble Q_post (fixed order).
__global__ void k_assemble_dqpost(int64_t nnzq, const double* __restrict__ dq,
                                  const int64_t* __restrict__ cptr, const int32_t* __restrict__ cpair,
                                  const int32_t* __restrict__ arow, const double* __restrict__ aval,
                                  const double* __restrict__ da, const double* __restrict__ qeps,
                                  const double* __restrict__ dqeps, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnzq;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = dq[e];
    for (int64_t c = cptr[e]; c < cptr[e + 1]; ++c) {
      const int32_t a1 = cpair[2 * c], a2 = cpair[2 * c + 1];
      const int32_t r = arow[a1];
      if (da) v += qeps[r] * (da[a1] * aval[a2] + aval[a1] * da[a2]);
      if (dqeps) v += dqeps[r] * aval[a1] * aval[a2];
    }
    out[e] = v;
  }
}

// out = base - V x over A's stored pattern with values V (m rows; base nullable = 0,
// base2 nullable, subtracted too); product_only != 0 writes V x itself
__global__ void k_spmv_obs(int64_t m, const int64_t* __restrict__ arp, const int32_t* __restrict__ aci,
                           const double* __restrict__ v, const double* __restrict__ x,
                           const double* __restrict__ base, const double* __restrict__ base2, int product_only,
                           double* __restrict__ out) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t e = arp[r]; e < arp[r + 1]; ++e) s += v[e] * x[aci[e]];
    double o = base ? base[r] : 0.0;
    if (base2) o -= base2[r];
    out[r] = product_only ? s : o - s;
  }
}

// elementwise: mode 0 out = a * b, 1 out = a / b, 2 out = log(a), 3 out = sqrt(a) * b
__global__ void k_elementwise(int64_t n, int mode, const double* __restrict__ a, const double* __restrict__ b,
                              double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = mode == 0 ? a[i] * b[i] : mode == 1 ? a[i] / b[i] : mode == 2 ? log(a[i]) : sqrt(a[i]) * b[i];
}

// ---- conjugate gradients (Sec. 3.2, CG method) with device scalars ----
// sc[0] = r^T z, sc[1] = p^T q, sc[2] = new r^T z
__global__ void k_cg_xr(int64_t n, const double* __restrict__ sc, const double* __restrict__ p,
                        const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r) {
  const double alpha = sc[1] != 0.0 ? sc[0] / sc[1] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
  }
}
__global__ void k_cg_p(int64_t n, double* __restrict__ sc, const double* __restrict__ z, double* __restrict__ p) {
  const double beta = sc[0] != 0.0 ? sc[2] / sc[0] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}
__global__ void k_cg_roll(double* __restrict__ sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc[0] = sc[2];
}
__global__ void k_copy_f64(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
// Jacobi: z = r / diag(Q)
__global__ void k_jacobi(int64_t n, const int64_t* __restrict__ qdiag, const double* __restrict__ qv,
                         const double* __restrict__ r, double* __restrict__ z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = r[i] / qv[qdiag[i]];
}

// Rao-Blackwellised variances from k draws x_s (n x k, column-major) of N(0, Q^-1):
// var_i = 1/Q_ii + (1/k) sum_s ((1/Q_ii) sum_{j != i} Q_ij x_sj)^2, fixed order
__global__ void k_rbmc(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       const double* __restrict__ qv, const int64_t* __restrict__ qdiag, int64_t k,
                       const double* __restrict__ xs, double* __restrict__ var) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ed = qdiag[i];
    const double d = qv[ed];
    double acc = 0.0;
    for (int64_t s2 = 0; s2 < k; ++s2) {
      const double* x = xs + s2 * n;
      double t = 0.0;
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
        if (e != ed) t += qv[e] * x[ci[e]];
      t /= d;
      acc += t * t;
    }
    var[i] = 1.0 / d + acc / (double)k;
  }
}

__global__ void k_obs_residual(int64_t m, const int64_t* __restrict__ arp, const int32_t* __restrict__ aci,
                               const double* __restrict__ aval, const double* __restrict__ qeps,
                               const double* __restrict__ y, const double* __restrict__ b,
                               const double* __restrict__ mu, double* __restrict__ rvec) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x) {
    double s = y[r];
    if (b) s -= b[r];
    if (mu) {
      double am = 0.0;
      for (int64_t e = arp[r]; e < arp[r + 1]; ++e) am += aval[e] * mu[aci[e]];
      s -= am;
    }
    rvec[r] = qeps[r] * s;
  }
}

__global__ void k_at_times(int64_t n, const int64_t* __restrict__ atp, const int32_t* __restrict__ ati,
                           const int32_t* __restrict__ arow, const double* __restrict__ aval,
                           const double* __restrict__ rvec, double* __restrict__ h) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t t = atp[i]; t < atp[i + 1]; ++t) {
      const int32_t a = ati[t];
      s += aval[a] * rvec[arow[a]];
    }
    h[i] = s;
  }
}

// power-of-two equilibration: s_i = 2^-floor(ilogb(Q_ii)/2), exact in floating point
__device__ __forceinline__ int eq_exp(double d) {
  if (!(d > 0.0) || !isfinite(d)) return 0;
  const int k = ilogb(d);
  return -(k >> 1);
}

__global__ void k_equil_rows(int64_t n, const int64_t* __restrict__ qdiag, const double* __restrict__ qpost,
                             int32_t* __restrict__ sexp, double* __restrict__ scale) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int e = eq_exp(qpost[qdiag[i]]);
    sexp[i] = e;
    scale[i] = ldexp(1.0, e);
  }
}

__global__ void k_equil_vals(int64_t nnzq, const int64_t* __restrict__ qdiag, const int32_t* __restrict__ qrow,
                             const int32_t* __restrict__ qcol, const double* __restrict__ qpost,
                             double* __restrict__ qhat) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnzq;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int er = eq_exp(qpost[qdiag[qrow[e]]]);
    const int ec = eq_exp(qpost[qdiag[qcol[e]]]);
    qhat[e] = ldexp(qpost[e], er + ec);
  }
}

template <typename V>
__global__ void k_fill(V* p, int64_t n, V v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Zero the lower triangle (diagonal included) of every listed front: work-group = 4
// consecutive columns.  The factorisation reads and writes only the lower triangles of the
// fronts, and the selected inversion writes every entry it reads.
constexpr int kZeroCols = 4;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero_lower(DevSym S, LaunchList L, T* __restrict__ W) {
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s);
  T* F = W + S.Woff[s];
#pragma unroll
  for (int q = 0; q < kZeroCols; ++q) {
    const int j = (int)loc * kZeroCols + q;
    if (j >= n) break;
    T* col = F + (int64_t)j * n;
    for (int i = j + threadIdx.x; i < n; i += kThreads) col[i] = T(0);
  }
}

template <typename T>
__global__ void k_scatter(int64_t cnt, const int64_t* __restrict__ map_e, const int64_t* __restrict__ map_off,
                          const double* __restrict__ qhat, T* __restrict__ W) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = map_e[i];
    if (e >= 0) W[map_off[i]] = (T)qhat[e];
  }
}

// ------------------------------------------------------------------ factorisation kernels
// child slot `slot` of every listed parent: add the child's update matrix (lower
// triangle, column `loc` per work-group) into the parent front.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_extend_add(DevSym S, LaunchList L, int slot,
                                                         const T* __restrict__ Wc, T* __restrict__ Wp) {
  // work-group: kExtCols consecutive columns b of the child's update matrix; each thread
  // loads a batch of relative row indices once and applies them to all of those columns
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int c = S.child_idx[S.child_ptr[s] + slot];
  const int nc = fn(S, c), pc = fp(S, c), uc = nc - pc;
  const int b0 = (int)loc * kExtCols;
  const int32_t* rel = S.relpos + S.rowptr[c] + pc;
  const int ns = fn(S, s);
  const T* src0 = Wc + S.Woff[c] + (int64_t)pc * nc + pc;
  T* dstf = Wp + S.Woff[s];
  int64_t dcol[kExtCols];
#pragma unroll
  for (int q = 0; q < kExtCols; ++q) dcol[q] = (int64_t)rel[min(b0 + q, uc - 1)] * ns;
  for (int a0 = b0 + threadIdx.x; a0 < uc; a0 += kThreads * kExtUnroll) {
    int ra[kExtUnroll];
#pragma unroll
    for (int v = 0; v < kExtUnroll; ++v) ra[v] = rel[min(a0 + kThreads * v, uc - 1)];
    T sv[kExtCols][kExtUnroll], dv[kExtCols][kExtUnroll];
#pragma unroll
    for (int q = 0; q < kExtCols; ++q) {
      const T* src = src0 + (int64_t)min(b0 + q, uc - 1) * nc;
#pragma unroll
      for (int v = 0; v < kExtUnroll; ++v) {
        sv[q][v] = src[min(a0 + kThreads * v, uc - 1)];
        dv[q][v] = dstf[dcol[q] + ra[v]];
      }
    }
#pragma unroll
    for (int q = 0; q < kExtCols; ++q) {
      const int b = b0 + q;
#pragma unroll
      for (int v = 0; v < kExtUnroll; ++v) {
        const int a = a0 + kThreads * v;
        if (b < uc && a >= b && a < uc) dstf[dcol[q] + ra[v]] = dv[q][v] + sv[q][v];
      }
    }
  }
}

// 1/sqrt(d) for d > 0 (normal range): the hardware estimate refined by two Newton steps
// y <- y (3/2 - (d/2) y^2), each of which roughly doubles the number of correct bits
__device__ __forceinline__ double rsqrt_newton(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}

// FP64 Cholesky of the step-th 64x64 diagonal block of each listed front and the inverse
// of the resulting lower-triangular block, both held in registers: thread (ti, tl) owns
// rows ti + 16a and columns tl + 16b (a, b < 4) of the block and of its inverse X.  Each
// phase j needs one barrier: the owners of column j (16 lanes of one wave, so the pivot is
// a lane read) finish it and publish it through LDS with zeros on and above the diagonal,
// which lets every thread apply the previous column to all its elements without
// predicates; the inverse follows two phases behind (forward substitution L X = I: row
// j-1 of X is scaled and published, row j-2 applied).  The phases are generated per
// 16-column block JB so that every register index is a compile-time constant.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int A>
__device__ __forceinline__ void potrf_scale_row(double (&x_r)[4][4], double* rowb, int tl, double rinv) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    x_r[A][b] *= rinv;
    rowb[tl + 16 * b] = x_r[A][b];
  }
}

template <int JB>
__device__ __forceinline__ void potrf_phase(int jr, int kb, int t, int ti, int tl, double (&a_r)[4][4],
                                            double (&x_r)[4][4], double (*colb)[kNB], double (*rowb)[kNB],
                                            double* pinv, int* fail) {
  const int j = 16 * JB + jr;
  if (j >= kb + 2) return;
  __syncthreads();
  // the owners of column j need only their column JB of the previous column's update
  // before they take the pivot: that part first, then the pivot, then the rest of the
  // phase's work (the other columns, the inverse), off the chain from barrier to barrier
  constexpr int B0 = JB < 4 ? JB : 0;
  const bool upd1 = j >= 1 && j - 1 < kb;
  double ci[4], cl[4];
  if (upd1) {
    const double* c1 = colb[(j - 1) & 3];
#pragma unroll
    for (int a = 0; a < 4; ++a) { ci[a] = c1[ti + 16 * a]; cl[a] = c1[tl + 16 * a]; }
#pragma unroll
    for (int a = 0; a < 4; ++a) a_r[a][B0] -= ci[a] * cl[B0];
  }
  if constexpr (JB < 4) {
    if (j < kb && (t >> 6) == (jr >> 2)) {
      double cv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) cv[a] = a_r[a][JB];
      const double d = readlane_f64(cv[JB], 16 * (jr & 3) + jr);
      if (tl == jr) {
        const bool bad = !(d > 0.0);
        const double linv = bad ? 1.0 : rsqrt_newton(d);
        const double ljj = bad ? 1.0 : d * linv;
        if (ti == jr) {
          pinv[j & 3] = linv;
          if (bad) atomicMin(fail, j);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = ti + 16 * a;
          const double v = i > j ? cv[a] * linv : 0.0;
          colb[j & 3][i] = v;
          a_r[a][JB] = i == j ? ljj : v;
        }
      }
    }
  }
  if (upd1) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b != B0) a_r[a][b] -= ci[a] * cl[b];
  }
  if (j >= 2 && j - 2 < kb) {
    const double* c2 = colb[(j - 2) & 3];
    const double* r2 = rowb[(j - 2) & 3];
    double ci[4], rc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) { ci[a] = c2[ti + 16 * a]; rc[a] = r2[tl + 16 * a]; }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) x_r[a][b] -= ci[a] * rc[b];
  }
  if (j >= 1 && j - 1 < kb && ti == ((j - 1) & 15)) {
    const double rinv = pinv[(j - 1) & 3];
    if (jr >= 1) {
      if constexpr (JB < 4) potrf_scale_row<JB>(x_r, rowb[(j - 1) & 3], tl, rinv);
    } else {
      if constexpr (JB >= 1) potrf_scale_row<JB - 1>(x_r, rowb[(j - 1) & 3], tl, rinv);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_potrf(DevSym S, LaunchList L, int step, NumBufs<T> B) {
  __shared__ double colb[4][kNB];
  __shared__ double rowb[4][kNB];
  __shared__ double pinv[4];
  __shared__ int fail;
  const int s = L.fronts[blockIdx.x];
  const int n = fn(S, s), p = fp(S, s);
  const int k0 = step * kNB;
  const int kb = min(kNB, p - k0);
  // a front of at most 64 rows is factored whole: its kb = p pivots are taken and the
  // rest of the block receives their update, so the panel below the diagonal block and
  // the update matrix come out of the same registers (no separate TRSM or SYRK)
  const int nbk = (step == 0 && n <= kNB) ? n : kb;
  T* F = B.Wcur + S.Woff[s];
  const int t = threadIdx.x, ti = t & 15, tl = t >> 4;
  double a_r[4][4], x_r[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ti + 16 * a, l = tl + 16 * b;
      const double v = (double)F[(k0 + min(i, nbk - 1)) + (int64_t)(k0 + min(l, nbk - 1)) * n];
      a_r[a][b] = (i < nbk && l < nbk && i >= l) ? v : 0.0;
      x_r[a][b] = i == l ? 1.0 : 0.0;
    }
  if (t == 0) fail = INT_MAX;
  for (int jr = 0; jr < 16; ++jr) potrf_phase<0>(jr, kb, t, ti, tl, a_r, x_r, colb, rowb, pinv, &fail);
  for (int jr = 0; jr < 16; ++jr) potrf_phase<1>(jr, kb, t, ti, tl, a_r, x_r, colb, rowb, pinv, &fail);
  for (int jr = 0; jr < 16; ++jr) potrf_phase<2>(jr, kb, t, ti, tl, a_r, x_r, colb, rowb, pinv, &fail);
  for (int jr = 0; jr < 16; ++jr) potrf_phase<3>(jr, kb, t, ti, tl, a_r, x_r, colb, rowb, pinv, &fail);
  for (int jr = 0; jr < 2; ++jr) potrf_phase<4>(jr, kb, t, ti, tl, a_r, x_r, colb, rowb, pinv, &fail);
  __syncthreads();
  T* Dblk = B.D + S.Doff[s] + (int64_t)step * kNB * kNB;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ti + 16 * a, l = tl + 16 * b;
      const bool in = i < kb && l < kb && i >= l;
      if (i < nbk && l < nbk && i >= l) F[(k0 + i) + (int64_t)(k0 + l) * n] = (T)a_r[a][b];
      Dblk[i + l * kNB] = in ? (T)x_r[a][b] : T(0);
      if (in && i == l) B.piv[S.sfirst[s] + k0 + i] = a_r[a][b];
    }
  if (t == 0 && fail != INT_MAX) atomicMin(B.status, S.sfirst[s] + k0 + fail);
}

// panel rows below the step-th diagonal block: F[r, blk] = F[r, blk] * Linv^T
template <typename T>
__global__ __launch_bounds__(kThreads) void k_trsm(DevSym S, LaunchList L, int step, NumBufs<T> B) {
  __shared__ T sA[kTile64Lds];
  __shared__ T sB[kTile64Lds];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const int k0 = step * kNB, kb = min(kNB, p - k0);
  const int row0 = k0 + kb + kTile * (int)loc;
  const int M = min(kTile, n - row0);
  T* F = B.Wcur + S.Woff[s];
  const T* Dblk = B.D + S.Doff[s] + (int64_t)step * kNB * kNB;
  typename V4<T>::type acc[2][2];
  zero_acc<T>(acc);
  gemm_tile<T, false, false>(F + row0 + (int64_t)k0 * n, n, Dblk, kNB, M, kb, kb, acc, sA, sB);
  for_acc<T>(acc, [&](int r, int c, T v) {
    if (r < M && c < kb) F[(row0 + r) + (int64_t)(k0 + c) * n] = v;
  });
}

// Lower-trapezoid tile update C -= A B^T inside each front: columns [clo, chi), rows
// from the column to n, reduction over front columns [klo, khi).  Two-level blocking:
//   mode 0 (inner, after 64-block `step`): columns up to the end of its 256-wide outer
//          block, K = the 64-block;
//   mode 1 (outer, after the last 64-block of an outer block): every panel column right
//          of the outer block, K = the 256-wide outer block;
//   mode 2 (SYRK): the update matrix, columns [p, n), K = all p pivot columns.
__device__ __forceinline__ void upd_region(int mode, int step, int n, int p, int& clo, int& chi,
                                           int& klo, int& khi) {
  if (mode == 2) { clo = p; chi = n; klo = 0; khi = p; return; }
  if (mode == 1) {
    const int k2 = (step / kSub) * kNB2;
    clo = k2 + kNB2; chi = p; klo = k2; khi = k2 + kNB2;
    return;
  }
  const int k0 = step * kNB, kb = min(kNB, p - k0);
  const int oe = min((step / kSub + 1) * kNB2, p);
  clo = k0 + kb; chi = oe; klo = k0; khi = k0 + kb;
}

// At least two work-groups per SIMD set: the FP64 instance otherwise takes 189+ VGPRs and
// all 128 AGPRs for one wave per SIMD, which leaves the FP64 matrix cores idle behind each
// chunk's loads (FP64 factor of the 1M-unknown space-time posterior: 931 -> 718 ms).
template <typename T, int TS>
__global__ __launch_bounds__(kThreads, 2) void k_update(DevSym S, LaunchList L, int step, int mode,
                                                     NumBufs<T> B) {
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  int clo, chi, klo, khi;
  upd_region(mode, step, n, p, clo, chi, klo, khi);
  int ct = 0;
  int64_t r = loc;
  while (true) {
    const int c0 = clo + TS * ct;
    if (c0 >= chi) return;   // unreachable for a consistent launch list
    const int64_t nr = (n - c0 + TS - 1) / TS;
    if (r < nr) break;
    r -= nr;
    ++ct;
  }
  const int col0 = clo + TS * ct;
  const int row0 = col0 + TS * (int)r;
  const int M = min(TS, n - row0), N = min(TS, chi - col0);
  T* F = B.Wcur + S.Woff[s];
  if constexpr (TS == 64) {
    __shared__ T sA[kTile64Lds];
    __shared__ T sB[kTile64Lds];
    typename V4<T>::type acc[2][2];
    zero_acc<T>(acc);
    gemm_tile<T, false, false>(F + row0 + (int64_t)klo * n, n, F + col0 + (int64_t)klo * n, n, M, N,
                               khi - klo, acc, sA, sB);
    acc_sub_lower<T, 2>(acc, F, n, row0, col0, M, N);
  } else {
    __shared__ __attribute__((aligned(16))) T sA[BigLds<T>::v];
    __shared__ __attribute__((aligned(16))) T sB[BigLds<T>::v];
    typename V4<T>::type acc[4][4];
    zero_acc128<T>(acc);
    gemm_tile128<T, false, false>(F + row0 + (int64_t)klo * n, n, F + col0 + (int64_t)klo * n, n, M, N,
                                  khi - klo, acc, sA, sB);
    acc_sub_lower<T, 4>(acc, F, n, row0, col0, M, N);
  }
}

// FP32 trailing SYRK (the update matrix: columns [p, n), K = all p pivot columns) in
// 256 x 256 tiles: 256-wide column tiles, rows from the tile's first column down.
__global__ __launch_bounds__(kThreads4, 1) void k_syrk4(DevSym S, LaunchList L, NumBufs<float> B) {
  __shared__ G4Smem sm;
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  int ct = 0;
  int64_t r = loc;
  while (true) {
    const int c0 = p + kG4 * ct;
    if (c0 >= n) return;   // unreachable for a consistent launch list
    const int64_t nr = (n - c0 + kG4 - 1) / kG4;
    if (r < nr) break;
    r -= nr;
    ++ct;
  }
  const int col0 = p + kG4 * ct;
  const int row0 = col0 + kG4 * (int)r;
  const int M = min(kG4, n - row0), N = min(kG4, n - col0);
  float* F = B.Wcur + S.Woff[s];
  f16v_t acc[4][2];
  zero_acc6(acc);
  gemm_tile4(F + row0, n, F + col0, n, M, N, p, acc, sm.g);
  g4_epilogue_sub(acc, sm, F, n, row0, col0, M, N);
}

// a[u] = sum over q = 0 .. split-1, in that order, of p[q PT + e0 + u stride] (u < U):
// four partials of U elements are loaded before they are added, so that 4 U independent
// loads are in flight per thread.
template <typename T, int U>
__device__ __forceinline__ void sum_parts(const T* __restrict__ p, int64_t PT, int split, int e0, int stride,
                                          T (&a)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = T(0);
  const T* pe = p + e0;
  int q = 0;
  for (; q + 4 <= split; q += 4) {
    T v[4][U];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int u = 0; u < U; ++u) v[j][u] = pe[(int64_t)(q + j) * PT + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] += v[0][u];
      a[u] += v[1][u];
      a[u] += v[2][u];
      a[u] += v[3][u];
    }
  }
  for (; q < split; ++q) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = pe[(int64_t)q * PT + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] += v[u];
  }
}

// FP32 left-looking update of outer block K of the pivot panel: before its first 64-block
// is factored, the block's columns [k2, k2 + kb2) (rows k2..n) receive
// -L[rows, 0:k2] L[cols, 0:k2]^T from all earlier outer blocks in one long-K product
// (256 x 256 tiles, one per 256 rows; split over K like the Sigma[R', K] products when a
// depth has too few tiles).  With split 1 the tile is subtracted in place (lower part
// only), else its partial goes to part + wg * 256^2 and k_panel_red4 subtracts the sum.
__global__ __launch_bounds__(kThreads4, 1) void k_panel_upd4(DevSym S, LaunchList L, int K, NumBufs<float> B,
                                                          float* __restrict__ part) {
  __shared__ G4Smem sm;
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const int k2 = K * kNB2, kb2 = min(kNB2, p - k2);
  const int split = L.aux[2 * fi];
  const int rt = (int)(loc / split), sp = (int)(loc % split);
  const int row0 = k2 + kG4 * rt;
  const int M = min(kG4, n - row0), N = kb2;
  const int kpart = ((k2 + split - 1) / split + kG4K - 1) / kG4K * kG4K;
  const int kb = min(k2, sp * kpart), ke = min(k2, kb + kpart);
  float* F = B.Wcur + S.Woff[s];
  f16v_t acc[4][2];
  zero_acc6(acc);
  gemm_tile4(F + row0 + (int64_t)kb * n, n, F + k2 + (int64_t)kb * n, n, M, N, ke - kb, acc, sm.g);
  if (split == 1) {
    g4_epilogue_sub(acc, sm, F, n, row0, k2, M, N);
  } else {
    float* out = part + wg_id() * (int64_t)(kG4 * kG4);
    g4_epilogue<false>(acc, sm, [&](int r, int c, float v) { out[r + c * kG4] = v; }, [](int, int, float) {});
  }
}

// Subtract the fixed-order sum of the split-K partials of k_panel_upd4 (one work-group per
// 64-column group of a tile; aux = (split, first work-group of the front in that launch)).
__global__ __launch_bounds__(kThreads) void k_panel_red4(DevSym S, LaunchList L, int K, NumBufs<float> B,
                                                         const float* __restrict__ part) {
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const int k2 = K * kNB2, kb2 = min(kNB2, p - k2);
  const int split = L.aux[2 * fi];
  const int64_t base = L.aux[2 * fi + 1];
  const int tile = (int)(loc >> 2), quarter = (int)(loc & 3);
  const int row0 = k2 + kG4 * tile, col0 = k2 + 64 * quarter;
  const int M = min(kG4, n - row0), N = min(64, k2 + kb2 - col0);
  if (N <= 0) return;
  constexpr int64_t PT = (int64_t)kG4 * kG4;
  const float* pp = part + (base + (int64_t)tile * split) * PT + (int64_t)(64 * quarter) * kG4;
  float* F = B.Wcur + S.Woff[s];
  constexpr int U = 8;
  for (int e0 = threadIdx.x; e0 < kG4 * 64; e0 += kThreads * U) {
    float a[U], old[U];
    sum_parts<float, U>(pp, PT, split, e0, kThreads, a);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kThreads, r = min(e % kG4, M - 1), c = min(e / kG4, N - 1);
      old[u] = F[(row0 + r) + (int64_t)(col0 + c) * n];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kThreads, r = e % kG4, c = e / kG4;
      const int gi = row0 + r, gj = col0 + c;
      if (r < M && c < N && gi >= gj) F[gi + (int64_t)gj * n] = old[u] - a[u];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_copy_L(DevSym S, LaunchList L, NumBufs<T> B) {
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s);
  const int j = (int)loc;
  const T* src = B.Wcur + S.Woff[s] + (int64_t)j * n;
  T* dst = B.L + S.Loff[s] + (int64_t)j * n;
  for (int i = j + threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// per-block log det = 2 sum log L^_jj - 2 ln2 sum e_i (equilibration exponents), summed
// in a fixed order: work-group (block, g) reduces its share of the block's pivots
// (strided per-thread sums, then a binary tree); a second pass adds the kLdParts partials
__global__ __launch_bounds__(kThreads) void k_logdet(const int64_t* __restrict__ bptr,
                                                     const int32_t* __restrict__ bpiv,
                                                     const int32_t* __restrict__ perm,
                                                     const double* __restrict__ piv,
                                                     const int32_t* __restrict__ sexp,
                                                     double* __restrict__ part) {
  __shared__ double red[kThreads];
  const int b = blockIdx.x / kLdParts, g = blockIdx.x % kLdParts;
  const int64_t q0 = bptr[b], len = bptr[b + 1] - q0;
  const int64_t per = (len + kLdParts - 1) / kLdParts;
  const int64_t lo = q0 + per * g, hi = min(bptr[b + 1], lo + per);
  double acc = 0.0;
  for (int64_t q = lo + threadIdx.x; q < hi; q += kThreads) {
    const int32_t j = bpiv[q];
    acc += 2.0 * log(piv[j]) - 2.0 * 0.69314718055994530942 * (double)sexp[perm[j]];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_logdet_final(int64_t nblocks, const double* __restrict__ part, double* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  double acc = 0.0;
  for (int g = 0; g < kLdParts; ++g) acc += part[b * kLdParts + g];
  out[b] = acc;
}

// ------------------------------------------------------------------ solve kernels
// front vector of supernode s: V + Voff[s]*nrhs, entry (i, r) at i + r*n_s
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fvec_init(DevSym S, LaunchList L, SolveBufs V) {
  const int s = L.fronts[blockIdx.x];
  const int n = fn(S, s), p = fp(S, s);
  double* v = V.Vcur + S.Voff[s] * V.nrhs;
  const int64_t f0 = S.sfirst[s];
  for (int idx = threadIdx.x; idx < n * V.nrhs; idx += blockDim.x) {
    const int i = idx % n, r = idx / n;
    v[idx] = i < p ? V.xp[f0 + i + (int64_t)r * S.n] : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fvec_extend(DevSym S, LaunchList L, int slot, SolveBufs V) {
  const int s = L.fronts[blockIdx.x];
  const int c = S.child_idx[S.child_ptr[s] + slot];
  const int nc = fn(S, c), pc = fp(S, c), uc = nc - pc;
  const int ns = fn(S, s);
  const int32_t* rel = S.relpos + S.rowptr[c] + pc;
  double* vp = V.Vcur + S.Voff[s] * V.nrhs;
  const double* vc = V.Vchild + S.Voff[c] * V.nrhs;
  for (int idx = threadIdx.x; idx < uc * V.nrhs; idx += blockDim.x) {
    const int a = idx % uc, r = idx / uc;
    vp[rel[a] + r * ns] += vc[pc + a + r * nc];
  }
}

// ---- solves blocked by 256-wide outer blocks ----
// The top separators turn the solves into a chain of short launches, so each launch is
// latency bound: every kernel keeps batches of 16-32 independent loads in flight per
// lane, and LDS is sized for NR right-hand sides (NR = 1, or 16 for the general case,
// nrhs <= NR) so that the many small fronts of the deep levels run at full occupancy.
template <int NR> struct RhsPad { static constexpr int v = NR == 1 ? 1 : NR + 1; };

// Forward, diagonal block of outer block t (left to right): x_K = Linv_KK v_K with the
// stored inverse.  Work-group (front, g) computes rows 64g..64g+63; its four waves take a
// quarter of the columns each and add their sums in a fixed order.  x_K goes to the
// pivot-order vector only, because the other work-groups of the launch still read v_K.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_fwd_block(DevSym S, LaunchList L, int t, const T* __restrict__ D2,
                                                        const int64_t* __restrict__ D2off, SolveBufs V) {
  constexpr int NP = RhsPad<NR>::v;
  __shared__ double xv[kNB2 * NR];
  __shared__ double red[kThreads * NP];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi], g = (int)loc;
  const int n = fn(S, s), p = fp(S, s);
  const int nr = NR == 1 ? 1 : V.nrhs;
  const int k2 = t * kNB2, kb2 = min(kNB2, p - k2);
  const int lend = 64 * g + 64;
  const double* v = V.Vcur + S.Voff[s] * nr;
  const T* X = D2 + D2off[s] + (int64_t)t * kNB2 * kNB2;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int i = 64 * g + lane;
  // NR = 1: the wave's 64 inverse entries are requested before the right-hand side is
  // staged, so that both memory round trips overlap
  T xr[NR == 1 ? 64 : 1];
  if constexpr (NR == 1) {
    // the stored inverse is zero above its diagonal, so only the block edges need masks
    const bool act = q <= g && i < kb2;
    const int ic = min(i, kb2 - 1);
#pragma unroll
    for (int u = 0; u < 64; ++u) {
      const int l = 64 * q + u;
      const T x = X[ic + (int64_t)min(l, kb2 - 1) * kb2];
      xr[u] = x * (T)(act && l < kb2);   // a product, not a select: keeps the load unconditional
    }
  }
  for (int idx = threadIdx.x; idx < lend * nr; idx += kThreads) {
    const int l = idx % lend, r = idx / lend;
    xv[l + r * kNB2] = l < kb2 ? v[k2 + l + (int64_t)r * n] : 0.0;
  }
  __syncthreads();
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  if constexpr (NR == 1) {
    if (q <= g) {
#pragma unroll
      for (int u = 0; u < 64; ++u) acc[0] += (double)xr[u] * xv[64 * q + u];
    }
  } else if (q <= g && i < kb2) {
    for (int l0 = 64 * q; l0 < 64 * q + 64; l0 += 16) {
      double xl[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) xl[u] = l0 + u <= i ? (double)X[i + (int64_t)(l0 + u) * kb2] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) acc[r] += xl[u] * xv[l0 + u + r * kNB2];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) red[threadIdx.x * NP + r] = acc[r];
  __syncthreads();
  if (q == 0 && i < kb2) {
    for (int r = 0; r < nr; ++r)
      V.xp[S.sfirst[s] + k2 + i + (int64_t)r * S.n] = (red[lane * NP + r] + red[(64 + lane) * NP + r]) +
                                                      (red[(128 + lane) * NP + r] + red[(192 + lane) * NP + r]);
  }
}

// Forward, rows below outer block t: v[rows] -= L[rows, K] x_K; 64 rows per work-group,
// the 256 columns split over the 4 waves and reduced through LDS.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_fwd_outer(DevSym S, LaunchList L, int t, const T* __restrict__ Lp,
                                                        SolveBufs V) {
  constexpr int NP = RhsPad<NR>::v;
  __shared__ double xs[kNB2 * NR];
  __shared__ double red[kThreads * NP];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const int nr = NR == 1 ? 1 : V.nrhs;
  const int k2 = t * kNB2, kb2 = min(kNB2, p - k2);
  const int64_t f0 = S.sfirst[s];
  double* v = V.Vcur + S.Voff[s] * nr;
  const int i = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int row = k2 + kb2 + 64 * (int)loc + i;
  const int c0 = cg * 64, c1 = min(kb2, c0 + 64);
  const T* Lr = Lp + S.Loff[s] + row + (int64_t)k2 * n;
  // NR = 1: all 64 column loads of the thread are in flight at once, requested before x_K
  // is staged (rows past n and columns past kb2 read as zero)
  T lv[NR == 1 ? 64 : 1];
  if constexpr (NR == 1) {
    const T* Lc = Lp + S.Loff[s] + min(row, n - 1) + (int64_t)k2 * n;
#pragma unroll
    for (int u = 0; u < 64; ++u) {
      const T x = Lc[(int64_t)min(c0 + u, kb2 - 1) * n];
      lv[u] = x * (T)(row < n && c0 + u < c1);
    }
  }
  for (int idx = threadIdx.x; idx < kNB2 * nr; idx += kThreads) {
    const int ii = idx % kNB2, r = idx / kNB2;
    xs[ii + r * kNB2] = ii < kb2 ? V.xp[f0 + k2 + ii + (int64_t)r * S.n] : 0.0;
  }
  __syncthreads();
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  if constexpr (NR == 1) {
#pragma unroll
    for (int u = 0; u < 64; ++u) acc[0] += (double)lv[u] * xs[c0 + u];
  } else if (row < n) {
    for (int cb = c0; cb < c1; cb += 16) {
      double lv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) lv[u] = cb + u < c1 ? (double)Lr[(int64_t)(cb + u) * n] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) acc[r] += lv[u] * xs[cb + u + r * kNB2];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) red[threadIdx.x * NP + r] = acc[r];
  __syncthreads();
  if (cg == 0 && row < n) {
    for (int r = 0; r < nr; ++r)
      v[row + (int64_t)r * n] -= (red[i * NP + r] + red[(64 + i) * NP + r]) +
                                 (red[(128 + i) * NP + r] + red[(192 + i) * NP + r]);
  }
}

// Backward split-K partials for outer block t (from the right): work-group (front,
// chunk of 256 rows below the block) computes part = L[chunk, K]^T x[chunk] (256 x nrhs);
// the front's first work-group also subtracts the right-hand side y_K, so that
// r_K = -(sum of the front's partials).
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_bwd_part(DevSym S, LaunchList L, int t, const T* __restrict__ Lp,
                                                       SolveBufs V, double* __restrict__ part) {
  // The x values of the work-group's 256 rows are gathered once into LDS; the L chunks
  // (32 rows x 256 columns) are software-pipelined: the next chunk's loads are issued
  // before the current chunk is multiplied, so one memory round trip stays exposed.
  constexpr int NP = RhsPad<NR>::v;
  __shared__ T Ls[32][kNB2 + 1];
  __shared__ double Xs[256 * NP];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const int nr = NR == 1 ? 1 : V.nrhs;
  const int nK = (p + kNB2 - 1) / kNB2, K = nK - 1 - t;
  const int k2 = K * kNB2, kb2 = min(kNB2, p - k2);
  const int rs = k2 + kb2;
  const int r0 = rs + 256 * (int)loc, r1 = min(n, r0 + 256);
  const int32_t* rows = S.rows + S.rowptr[s];
  const T* Lf = Lp + S.Loff[s];
  const int c = threadIdx.x;
  T tmp[32];
  auto load_chunk = [&](int i0) {
    const int mi = min(32, r1 - i0);
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int idx = threadIdx.x + k * kThreads;
      const int ii = idx & 31, cc = idx >> 5;
      const T x = Lf[(i0 + min(ii, mi - 1)) + (int64_t)(k2 + min(cc, kb2 - 1)) * n];
      tmp[k] = x * (T)(ii < mi && cc < kb2);
    }
  };
  if (r0 < r1) load_chunk(r0);
  for (int idx = threadIdx.x; idx < 256 * nr; idx += kThreads) {
    const int ii = idx & 255, r = idx >> 8;
    Xs[ii * NP + r] = r0 + ii < r1 ? V.xp[rows[r0 + ii] + (int64_t)r * S.n] : 0.0;
  }
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  for (int i0 = r0; i0 < r1; i0 += 32) {
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int idx = threadIdx.x + k * kThreads;
      Ls[idx & 31][idx >> 5] = tmp[k];
    }
    if (i0 + 32 < r1) load_chunk(i0 + 32);
    __syncthreads();
    const double* xc = Xs + (i0 - r0) * NP;
#pragma unroll 8
    for (int ii = 0; ii < 32; ++ii) {
      const double l = (double)Ls[ii][c];
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r < nr) acc[r] += l * xc[ii * NP + r];
    }
    __syncthreads();
  }
  if (loc == 0 && c < kb2) {
    const int64_t f0 = S.sfirst[s];
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nr) acc[r] -= V.xp[f0 + k2 + c + (int64_t)r * S.n];
  }
  // only the block's kb2 columns are read back (small fronts have few)
  double* out = part + wg_id() * (int64_t)(kNB2 * 16);
  if (c < kb2) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nr) out[c + r * kNB2] = acc[r];
  }
}

// Backward, diagonal block from the right: r_K = -(sum of the partials) and
// x_K = Linv_KK^T r_K, read from the stored transpose XT of the inverse so that lanes
// walk rows.  Work-group (front, g) computes x for columns 64g..64g+63: it first forms
// r_l for l >= 64g (the threads splitting the partials when fewer l remain), then the
// four waves take a quarter of l each.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_bwd_block(DevSym S, LaunchList L, LaunchList Lpart, int t,
                                                        const T* __restrict__ D2T,
                                                        const int64_t* __restrict__ D2off, SolveBufs V,
                                                        const double* __restrict__ part) {
  constexpr int NP = RhsPad<NR>::v;
  __shared__ double rv[kNB2 * NR];
  __shared__ double red[kThreads * NP];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi], g = (int)loc;
  const int p = fp(S, s);
  const int nr = NR == 1 ? 1 : V.nrhs;
  const int nK = (p + kNB2 - 1) / kNB2, K = nK - 1 - t;
  const int k2 = K * kNB2, kb2 = min(kNB2, p - k2);
  const int64_t f0 = S.sfirst[s];
  const int64_t q0 = Lpart.prefix[fi], q1 = Lpart.prefix[fi + 1];
  const T* XT = D2T + D2off[s] + (int64_t)K * kNB2 * kNB2;
  const int l0 = 64 * g;
  const int nch = (kb2 - l0 + 63) / 64;           // 1..4 chunks of l
  const int split = 4 / nch;                      // threads per l
  const int span = 64 * nch;
  const int li = threadIdx.x % span, pid = threadIdx.x / span;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int i = l0 + lane;
  // NR = 1: the wave's 64 entries of the transposed inverse are requested first (they do
  // not depend on r), and the partials are summed in batches of 32 loads in flight
  T xt[NR == 1 ? 64 : 1];
  if constexpr (NR == 1) {
    // the stored transpose is zero below its diagonal, so only the block edges need masks
    const bool act = q >= g && 64 * q < kb2 && i < kb2;
    const int ic = min(i, kb2 - 1);
#pragma unroll
    for (int u = 0; u < 64; ++u) {
      const int l = 64 * q + u;
      const T x = XT[ic + (int64_t)min(l, kb2 - 1) * kb2];
      xt[u] = x * (T)(act && l < kb2);
    }
  }
  {
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    const int l = l0 + li;
    if (NR == 1 && pid < split && l < kb2) {
      for (int64_t qb = q0 + pid; qb < q1; qb += (int64_t)split * 32) {
        double w[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int64_t qq = qb + (int64_t)u * split;
          const double x = part[min(qq, q1 - 1) * (kNB2 * 16) + l];
          w[u] = x * (double)(qq < q1);
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) acc[0] += w[u];
      }
    } else if (pid < split && l < kb2) {
#pragma unroll 8
      for (int64_t q = q0 + pid; q < q1; q += split) {
        const double* pq = part + q * (kNB2 * 16) + l;
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) acc[r] += pq[r * kNB2];
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) red[threadIdx.x * NP + r] = acc[r];
    __syncthreads();
    if (pid == 0) {
      for (int r = 0; r < nr; ++r) {
        double a = red[li * NP + r];
        for (int pp = 1; pp < split; ++pp) a += red[(pp * span + li) * NP + r];
        rv[l + r * kNB2] = l < kb2 ? -a : 0.0;
      }
    }
    __syncthreads();
  }
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  if constexpr (NR == 1) {
    if (q >= g && 64 * q < kb2) {
#pragma unroll
      for (int u = 0; u < 64; ++u) acc[0] += (double)xt[u] * rv[64 * q + u];
    }
  } else if (q >= g && 64 * q < kb2 && i < kb2) {
    for (int lb = 64 * q; lb < 64 * q + 64; lb += 16) {
      double xl[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int l = lb + u;
        xl[u] = (l >= i && l < kb2) ? (double)XT[i + (int64_t)l * kb2] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) acc[r] += xl[u] * rv[lb + u + r * kNB2];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) red[threadIdx.x * NP + r] = acc[r];
  __syncthreads();
  if (q == 0 && i < kb2) {
    for (int r = 0; r < nr; ++r)
      V.xp[f0 + k2 + i + (int64_t)r * S.n] = (red[lane * NP + r] + red[(64 + lane) * NP + r]) +
                                             (red[(128 + lane) * NP + r] + red[(192 + lane) * NP + r]);
  }
}

// xp = gate * S P src (gate == nullptr: factor 1); a zero gate turns the solve that
// follows into a no-op correction (converged refinement inside a captured sequence)
__global__ void k_permute_in(int64_t n, int nrhs, const int32_t* __restrict__ perm, const double* __restrict__ scale,
                             const double* __restrict__ src, int64_t lds, double* __restrict__ xp,
                             const double* __restrict__ gate) {
  const int64_t tot = n * nrhs;
  const double g = gate ? gate[0] : 1.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = q % n, r = q / n;
    const int32_t o = perm[j];
    xp[q] = g * (scale[o] * src[o + r * lds]);
  }
}

// Refinement gate on the device: norms[0] = ||h||, norms[1] = ||r||; gate[0] = 1 while
// ||r|| > tol ||h|| (the next correction is applied), else 0; gate[1] counts the applied
// corrections.  With record != 0 it writes the relative residual and that count instead.
__global__ void k_refine_gate(const double* __restrict__ norms, double tol, double* __restrict__ gate,
                              double* __restrict__ rec, int record) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double hn = norms[0] > 0.0 ? norms[0] : 1.0;
  const double rel = norms[1] / hn;
  if (record) {
    rec[0] = rel;
    rec[1] = gate[1];
    return;
  }
  const double g = (rel > tol || !(rel == rel)) ? 1.0 : 0.0;
  gate[0] = g;
  gate[1] += g;
}

__global__ void k_permute_in_f32(int64_t tot, const float* __restrict__ z, double* __restrict__ xp) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot;
       q += (int64_t)gridDim.x * blockDim.x)
    xp[q] = (double)z[q];
}

__global__ void k_permute_out(int64_t n, int nrhs, const int32_t* __restrict__ perm, const double* __restrict__ scale,
                              const double* __restrict__ xp, const double* __restrict__ add, int64_t ldadd,
                              double* __restrict__ out, int64_t ldo, int accumulate) {
  const int64_t tot = n * nrhs;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = q % n, r = q / n;
    const int32_t o = perm[j];
    double v = scale[o] * xp[q];
    if (accumulate) v += out[o + r * ldo];
    else if (add) v += add[o + r * ldadd];
    out[o + r * ldo] = v;
  }
}

// CSR rows of Q: a group of kRowG lanes per row, lane j summing entries j, j + kRowG, ...
// (coalesced, few dependent loads per lane), then a fixed butterfly over the group, so
// the sum order is the same on every call.
constexpr int kRowG = 16;
__device__ __forceinline__ double csr_row_dot(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                              const double* __restrict__ val, const double* __restrict__ x,
                                              int64_t i, int j) {
  double s = 0.0;
  const int64_t e1 = rp[i + 1];
  for (int64_t e = rp[i] + j; e < e1; e += kRowG) s += val[e] * x[ci[e]];
  s += __shfl_xor(s, 8, kRowG);
  s += __shfl_xor(s, 4, kRowG);
  s += __shfl_xor(s, 2, kRowG);
  s += __shfl_xor(s, 1, kRowG);
  return s;
}

__global__ void k_resid(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                        const double* __restrict__ val, const double* __restrict__ h,
                        const double* __restrict__ x, double* __restrict__ r) {
  const int j = threadIdx.x & (kRowG - 1);
  const int64_t gs = (int64_t)gridDim.x * blockDim.x / kRowG;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowG; i < n; i += gs) {
    const double s = csr_row_dot(rp, ci, val, x, i, j);
    if (j == 0) r[i] = h[i] - s;
  }
}

__global__ void k_add(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = b ? a[i] + b[i] : a[i];
}

// Whittle-Matern precision values on Q's pattern (alpha = 2):
// Q = tau^-2 (kappa^4 M~ + 2 kappa^2 S + S M~^-1 S) = tau^-2 K M~^-1 K with K = kappa^2 M~ + S,
// dQ/dlog(kappa) = 4 kappa^2 tau^-2 K
__global__ void k_matern_values(int64_t nnz, const double* __restrict__ mv, const double* __restrict__ sv,
                                const double* __restrict__ smsv, double kappa, double tau,
                                double* __restrict__ q, double* __restrict__ dq) {
  const double k2 = kappa * kappa, it2 = 1.0 / (tau * tau);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    q[e] = it2 * (k2 * k2 * mv[e] + 2.0 * k2 * sv[e] + smsv[e]);
    if (dq) dq[e] = 4.0 * k2 * it2 * (k2 * mv[e] + sv[e]);
  }
}

__global__ void k_spmv(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       const double* __restrict__ val, const double* __restrict__ x, double* __restrict__ y) {
  const int j = threadIdx.x & (kRowG - 1);
  const int64_t gs = (int64_t)gridDim.x * blockDim.x / kRowG;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowG; i < n; i += gs) {
    const double s = csr_row_dot(rp, ci, val, x, i, j);
    if (j == 0) y[i] = s;
  }
}

// w_r = sqrt(q_eps_r) (y_r - b_r - (A x)_r)
__global__ void k_weighted_resid(int64_t m, const int64_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                 const double* __restrict__ aval, const double* __restrict__ qeps,
                                 const double* __restrict__ y, const double* __restrict__ b,
                                 const double* __restrict__ x, double* __restrict__ w) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x) {
    double s = y[r];
    if (b) s -= b[r];
    for (int64_t e = arp[r]; e < arp[r + 1]; ++e) s -= aval[e] * x[aci[e]];
    w[r] = sqrt(qeps[r]) * s;
  }
}

// ---- Gauss-Newton for the Galerkin implicit-Euler Burgers residual (Sec. 3.3) ----
// Unknowns u^k_i at slice k (0..nt-1) and interior node i (0..nx-1), index k*nx + i;
// homogeneous Dirichlet values outside.  Rows of A: i (k = 0) observe u^0_i; row
// nx + (k-1)*nx + i (k >= 1) is the Galerkin residual
//   f = m_i (u^k_i - u^(k-1)_i)/dt + nu (S u^k)_i + B_i(u^k),
//   B_i(u) = (u_{i+1}^2 + u_i u_{i+1} - u_{i-1} u_i - u_{i-1}^2) / 6   (P1, exact quadrature of
//   the weak form of u u_x = (u^2/2)_x), stored as [(k-1)nx+i, k nx+i-1, k nx+i, k nx+i+1].
// B is quadratic, so the linearisation f(u) ~ J(u_bar) u + b has b = -B(u_bar).
__device__ __forceinline__ double burg_B(double um, double u0, double up) {
  return (up * up + u0 * up - um * u0 - um * um) * (1.0 / 6.0);
}

__global__ void k_burgers_linearize(int64_t nx, int64_t nt, double dt, double nu, const double* __restrict__ mass,
                                    const double* __restrict__ s3, const double* __restrict__ u,
                                    const int64_t* __restrict__ arp, double* __restrict__ aval,
                                    double* __restrict__ b) {
  const int64_t m = nx * nt;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = arp[r];
    if (r < nx) { aval[e] = 1.0; b[r] = 0.0; continue; }
    const int64_t q = r - nx, k = q / nx + 1, i = q % nx;
    const double* uk = u + k * nx;
    const double um = i > 0 ? uk[i - 1] : 0.0, u0 = uk[i], up = i + 1 < nx ? uk[i + 1] : 0.0;
    aval[e++] = -mass[i] / dt;
    if (i > 0) aval[e++] = nu * s3[3 * i] + (-u0 - 2.0 * um) * (1.0 / 6.0);
    aval[e++] = mass[i] / dt + nu * s3[3 * i + 1] + (up - um) * (1.0 / 6.0);
    if (i + 1 < nx) aval[e++] = nu * s3[3 * i + 2] + (2.0 * up + u0) * (1.0 / 6.0);
    b[r] = -burg_B(um, u0, up);
  }
}

// Residual of row r at u + alpha d (the nonlinear f, minus the data y)
__device__ __forceinline__ double burg_resid(int64_t r, int64_t nx, double dt, double nu,
                                             const double* __restrict__ mass, const double* __restrict__ s3,
                                             const double* __restrict__ u, const double* __restrict__ d,
                                             double alpha, const double* __restrict__ y) {
  if (r < nx) return (u[r] + alpha * d[r]) - y[r];
  const int64_t q = r - nx, k = q / nx + 1, i = q % nx;
  const int64_t c = k * nx + i, cp = (k - 1) * nx + i;
  auto U = [&](int64_t j) { return u[j] + alpha * d[j]; };
  const double um = i > 0 ? U(c - 1) : 0.0, u0 = U(c), up = i + 1 < nx ? U(c + 1) : 0.0;
  const double su = s3[3 * i] * um + s3[3 * i + 1] * u0 + s3[3 * i + 2] * up;
  return mass[i] * (u0 - U(cp)) / dt + nu * su + burg_B(um, u0, up) - y[r];
}

// partial sums for 9 trial step lengths alpha_j = 2^-j (j = 0..7) and alpha = 0 (index 8):
// part[j * kRedBlocksGN + block] = sum_r q_eps_r f_r(u + alpha_j d)^2; also the directional
// term part[9 * kRedBlocksGN + block] = sum_r q_eps_r f_r(u) (J d)_r with J from aval
constexpr int kRedBlocksGN = 256;
__global__ __launch_bounds__(256) void k_burgers_trials(int64_t nx, int64_t nt, double dt, double nu,
                                                        const double* __restrict__ mass, const double* __restrict__ s3,
                                                        const double* __restrict__ u, const double* __restrict__ d,
                                                        const double* __restrict__ y, const double* __restrict__ qeps,
                                                        const int64_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                                        const double* __restrict__ aval, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t m = nx * nt;
  double acc[10];
#pragma unroll
  for (int j = 0; j < 10; ++j) acc[j] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < m; r += (int64_t)kRedBlocksGN * 256) {
    const double w = qeps[r];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double f = burg_resid(r, nx, dt, nu, mass, s3, u, d, ldexp(1.0, -j), y);
      acc[j] += w * f * f;
    }
    const double f0 = burg_resid(r, nx, dt, nu, mass, s3, u, d, 0.0, y);
    acc[8] += w * f0 * f0;
    double jd = 0.0;
    for (int64_t e = arp[r]; e < arp[r + 1]; ++e) jd += aval[e] * d[aci[e]];
    acc[9] += w * f0 * jd;
  }
  for (int j = 0; j < 10; ++j) {
    red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[j * kRedBlocksGN + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// Sums the partials in a fixed order and picks the step: quad[0] = u^T Q u,
// quad[1] = u^T Q d, quad[2] = d^T Q d; phi(alpha) = 1/2 (u+ad)^T Q (u+ad) + 1/2 data(alpha);
// Armijo with c = 1e-4 on the first of alpha = 1, 1/2, ..., 1/128 that passes (none:
// alpha = 0, the step is not taken); writes alpha to sel[0] and the iteration record
// (phi0, alpha, decrement, slope) to rec[0..3].
__global__ void k_gn_select(const double* __restrict__ part, const double* __restrict__ quad,
                            double* __restrict__ sel, double* __restrict__ rec) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double data[10];
  for (int j = 0; j < 10; ++j) {
    double s = 0.0;
    for (int b = 0; b < kRedBlocksGN; ++b) s += part[j * kRedBlocksGN + b];
    data[j] = s;
  }
  const double uQu = quad[0], uQd = quad[1], dQd = quad[2];
  const double phi0 = 0.5 * uQu + 0.5 * data[8];
  const double slope = uQd + data[9];          // grad phi^T d
  // the first trial that passes the Armijo test; none: the step is not taken
  double alpha = 0.0;
  for (int j = 0; j < 8; ++j) {
    const double a = ldexp(1.0, -j);
    const double phi = 0.5 * (uQu + 2.0 * a * uQd + a * a * dQd) + 0.5 * data[j];
    if (phi <= phi0 + 1e-4 * a * slope) { alpha = a; break; }
  }
  sel[0] = alpha;
  rec[0] = phi0;
  rec[1] = alpha;
  rec[2] = -slope;                              // Newton decrement lambda^2 = -grad^T d
  rec[3] = slope;
}

// ---- Gauss-Newton for residuals with a pointwise power nonlinearity (Sec. 3.3) ----
// Row r: f_r(u) = sum_e lin[e] u[col e] + c_r u_j^p with j = nl_col[r] (-1: linear row),
// c_r = nl_coef[r]; the unknown j must be one of the row's stored columns.  Linearised at
// u: J = lin + p c u_j^(p-1) at column j, and f ~ J u + b with b = (1 - p) c u_j^p.
__device__ __forceinline__ double ipow(double x, int p) {
  double r = 1.0;
  for (int k = 0; k < p; ++k) r *= x;
  return r;
}

__global__ void k_pw_linearize(int64_t m, const int64_t* __restrict__ arp, const int32_t* __restrict__ aci,
                               const double* __restrict__ lin, const int32_t* __restrict__ nl_col,
                               const double* __restrict__ nl_coef, int power, const double* __restrict__ u,
                               double* __restrict__ aval, double* __restrict__ b) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = nl_col[r];
    const double c = j >= 0 ? nl_coef[r] : 0.0;
    const double uj = j >= 0 ? u[j] : 0.0;
    for (int64_t e = arp[r]; e < arp[r + 1]; ++e)
      aval[e] = lin[e] + (aci[e] == j ? (double)power * c * ipow(uj, power - 1) : 0.0);
    b[r] = (1.0 - (double)power) * c * ipow(uj, power);
  }
}

// partial sums for the trial steps alpha_j = 2^-j (j = 0..7) and alpha = 0 (index 8) of
// sum_r q_eps_r (f_r(u + alpha d) - y_r)^2, and the directional term sum_r q_eps_r
// (f_r(u) - y_r) (J d)_r (index 9), laid out like the Burgers line search
__global__ __launch_bounds__(256) void k_pw_trials(int64_t m, const int64_t* __restrict__ arp,
                                                   const int32_t* __restrict__ aci, const double* __restrict__ lin,
                                                   const int32_t* __restrict__ nl_col,
                                                   const double* __restrict__ nl_coef, int power,
                                                   const double* __restrict__ u, const double* __restrict__ d,
                                                   const double* __restrict__ y, const double* __restrict__ qeps,
                                                   const double* __restrict__ aval, double* __restrict__ part) {
  __shared__ double red[256];
  double acc[10];
#pragma unroll
  for (int j = 0; j < 10; ++j) acc[j] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < m; r += (int64_t)kRedBlocksGN * 256) {
    double lu = 0.0, ld = 0.0, jd = 0.0;
    for (int64_t e = arp[r]; e < arp[r + 1]; ++e) {
      const double ue = u[aci[e]], de = d[aci[e]];
      lu += lin[e] * ue;
      ld += lin[e] * de;
      jd += aval[e] * de;
    }
    const int32_t jn = nl_col[r];
    const double c = jn >= 0 ? nl_coef[r] : 0.0;
    const double uj = jn >= 0 ? u[jn] : 0.0, dj = jn >= 0 ? d[jn] : 0.0;
    const double w = qeps[r];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double a = ldexp(1.0, -k);
      const double f = lu + a * ld + c * ipow(uj + a * dj, power) - y[r];
      acc[k] += w * f * f;
    }
    const double f0 = lu + c * ipow(uj, power) - y[r];
    acc[8] += w * f0 * f0;
    acc[9] += w * f0 * jd;
  }
  for (int j = 0; j < 10; ++j) {
    red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[j * kRedBlocksGN + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// d = x - u (GN direction from the linearised posterior mean x); then u += sel[0] * d
__global__ void k_gn_direction(int64_t n, const double* __restrict__ x, const double* __restrict__ u,
                               double* __restrict__ d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = x[i] - u[i];
}
__global__ void k_gn_update(int64_t n, const double* __restrict__ sel, const double* __restrict__ d,
                            double* __restrict__ u) {
  const double a = sel[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    u[i] += a * d[i];
}

constexpr int kRedBlocks = 512;

// deterministic two-pass sum of a[i]*b[i] (b == nullptr: a[i]^2)
__global__ __launch_bounds__(kThreads) void k_dot_partial(int64_t n, const double* __restrict__ a,
                                                          const double* __restrict__ b,
                                                          double* __restrict__ partial) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kThreads)
    acc += a[i] * (b ? b[i] : a[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void k_dot_final(const double* __restrict__ partial, int sq,
                                                        double* __restrict__ out) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += kThreads) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sq ? sqrt(red[0]) : red[0];
}

// ---- Jacobi-preconditioned CG, five launches per iteration ----
// The streaming kernels run kCgBlocks work-groups (enough waves in flight for the gathers of
// the CSR product) with a fixed assignment of rows; each writes one partial sum per
// work-group, which a one-work-group kernel adds in a fixed order, so the iteration is
// deterministic.  sc holds r^T z of the current iteration in slot `cur` and receives the next
// one in slot 1 - cur; sc[2] receives p^T q, sc[5] the squared residual norm.
constexpr int kCgBlocks = 2048;
static_assert(kCgPartials == 3 * kCgBlocks, "CG partial buffer layout");

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// q = Q p (16 lanes per CSR row) and the partials of p^T q
__global__ __launch_bounds__(kThreads) void k_cg_spmv_pq(int64_t n, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ p, double* __restrict__ q,
                                                         double* __restrict__ part_pq) {
  __shared__ double red[kThreads];
  const int j = threadIdx.x & (kRowG - 1);
  const int64_t gs = (int64_t)kCgBlocks * kThreads / kRowG;
  double acc = 0.0;
  for (int64_t i = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kRowG; i < n; i += gs) {
    const double s = csr_row_dot(rp, ci, val, p, i, j);
    if (j == 0) {
      q[i] = s;
      acc += p[i] * s;
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part_pq[blockIdx.x] = t;
}

// out = sum of the kCgBlocks partials, in a fixed order (one work-group)
__global__ __launch_bounds__(kThreads) void k_cg_sum(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kCgBlocks; i += kThreads) acc += part[i];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = t;
}

// alpha = r^T z / p^T q; x += alpha p; r -= alpha q; z = r / diag(Q); partials of r^T z, r^T r
__global__ __launch_bounds__(kThreads) void k_cg_update(int64_t n, const double* __restrict__ sc, int cur,
                                                        const double* __restrict__ p, const double* __restrict__ q,
                                                        double* __restrict__ x, double* __restrict__ r,
                                                        const int64_t* __restrict__ qdiag,
                                                        const double* __restrict__ qv, double* __restrict__ z,
                                                        double* __restrict__ part_rz, double* __restrict__ part_rr) {
  __shared__ double red[kThreads];
  const double pq = sc[2];
  const double alpha = pq != 0.0 ? sc[cur] / pq : 0.0;
  double arz = 0.0, arr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)kCgBlocks * kThreads) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    const double zi = ri / qv[qdiag[i]];
    z[i] = zi;
    arz += ri * zi;
    arr += ri * ri;
  }
  const double trz = block_sum(arz, red);
  const double trr = block_sum(arr, red);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = trz;
    part_rr[blockIdx.x] = trr;
  }
}

__global__ void k_cg_sqrt(double* __restrict__ v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) v[0] = sqrt(v[2]);
}

// beta = new r^T z / r^T z; p = z + beta p
__global__ __launch_bounds__(kThreads) void k_cg_pupdate(int64_t n, const double* __restrict__ sc, int cur,
                                                         const double* __restrict__ z, double* __restrict__ p) {
  const double beta = sc[cur] != 0.0 ? sc[1 - cur] / sc[cur] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)kCgBlocks * kThreads)
    p[i] = z[i] + beta * p[i];
}

// ------------------------------------------------------------------ selected inversion
// Sigma front of s: square n_s x n_s (both triangles) at Scur + Woff[s].
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sel_gather(DevSym S, LaunchList L, const int32_t* __restrict__ sparent,
                                                          SelBufs<T> B) {
  // work-group: kExtCols consecutive columns of the child's Sigma_RR block, gathered from
  // the parent's square Sigma front through the relative indices (loaded once per batch)
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s), u = n - p;
  const int par = sparent[s];
  const int np = fn(S, par);
  const int b0 = (int)loc * kExtCols;
  const int32_t* rel = S.relpos + S.rowptr[s] + p;
  T* dst0 = B.Scur + S.Woff[s] + (int64_t)p * n + p;
  const T* srcf = B.Spar + S.Woff[par];
  int64_t scol[kExtCols];
#pragma unroll
  for (int q = 0; q < kExtCols; ++q) scol[q] = (int64_t)rel[min(b0 + q, u - 1)] * np;
  for (int a0 = threadIdx.x; a0 < u; a0 += kThreads * kExtUnroll) {
    int ra[kExtUnroll];
#pragma unroll
    for (int v = 0; v < kExtUnroll; ++v) ra[v] = rel[min(a0 + kThreads * v, u - 1)];
    T val[kExtCols][kExtUnroll];
#pragma unroll
    for (int q = 0; q < kExtCols; ++q)
#pragma unroll
      for (int v = 0; v < kExtUnroll; ++v) val[q][v] = srcf[scol[q] + ra[v]];
#pragma unroll
    for (int q = 0; q < kExtCols; ++q) {
      const int b = b0 + q;
      T* dst = dst0 + (int64_t)b * n;
#pragma unroll
      for (int v = 0; v < kExtUnroll; ++v) {
        const int a = a0 + kThreads * v;
        if (b < u && a < u) dst[a] = val[q][v];
      }
    }
  }
}

// ---- two-level selected inversion: 256-wide outer blocks K (counted from the right) ----
// For the outer block K of front s with rows after it R' (n' = n - k2 - kb2 rows):
//   X = L[R', K] Linv_KK,  Sigma[R', K] = -Sigma[R', R'] X,
//   Sigma[K, K] = Linv_KK^T Linv_KK - X^T Sigma[R', K]
// (the supernodal Takahashi relations with K as the supernode and R' its row set).
struct OuterBlk { int K, k2, kb2, rs, nsub; };
__device__ __forceinline__ OuterBlk outer_blk(int p, int n, int step) {
  OuterBlk o;
  const int nK = (p + kNB2 - 1) / kNB2;
  o.K = nK - 1 - step;
  o.k2 = o.K * kNB2;
  o.kb2 = min(kNB2, p - o.k2);
  o.rs = o.k2 + o.kb2;
  o.nsub = (o.kb2 + kNB - 1) / kNB;
  (void)n;
  return o;
}

// Inverse of every 256-wide outer diagonal block, Linv_KK = L_KK^-1, from the 64-block
// inverses: column block j of X = L_KK^-1 has X_jj = Linv_jj and
// X_ij = -Linv_ii sum_{j<=l<i} L_il X_lj for i > j.  One work-group per (front, 64-block
// b), b = 4 K + j; X is column-major with ld kb2 at D2 + D2off[s] + K * 256^2 (zeros
// above the diagonal).  `base` selects where L lives: the square front (during the
// factorisation) or the L panel storage; both have leading dimension n_s.  Each column
// block is written and read back by the same work-group only, so its barriers (work-group
// scope) order those stores; a device-scope fence here would write back the L2 cache in
// every one of the (many, on a forest of small fronts) work-groups.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_inv256(DevSym S, LaunchList L, const T* __restrict__ Lbase,
                                                     int from_front, const T* __restrict__ Dinv,
                                                     const int64_t* __restrict__ D2off, T* __restrict__ D2,
                                                     T* __restrict__ D2T) {
  __shared__ T sA[kTile64Lds];
  __shared__ T sB[kTile64Lds];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const int K = (int)(loc / kSub), j = (int)(loc % kSub);
  const int k2 = K * kNB2, kb2 = min(kNB2, p - k2);
  const int nsub = (kb2 + kNB - 1) / kNB;
  const int sbj = min(kNB, kb2 - kNB * j);
  T* X = D2 + D2off[s] + (int64_t)K * kNB2 * kNB2;
  T* XT = D2T + D2off[s] + (int64_t)K * kNB2 * kNB2;
  const T* Lf = Lbase + (from_front ? S.Woff[s] : S.Loff[s]);
  const int blk0 = k2 / kNB;
  for (int idx = threadIdx.x; idx < kb2 * kNB; idx += kThreads) {
    const int r = idx % kb2, c = idx / kb2;
    if (c < sbj) {
      T v = T(0);
      if (r >= kNB * j && r < kNB * j + sbj)
        v = Dinv[S.Doff[s] + (int64_t)(blk0 + j) * kNB * kNB + (r - kNB * j) + c * kNB];
      X[r + (int64_t)(kNB * j + c) * kb2] = v;
    }
  }
  for (int idx = threadIdx.x; idx < kb2 * sbj; idx += kThreads) {
    const int c = idx % sbj, r = idx / sbj;
    T v = T(0);
    if (r >= kNB * j && r < kNB * j + sbj)
      v = Dinv[S.Doff[s] + (int64_t)(blk0 + j) * kNB * kNB + (r - kNB * j) + c * kNB];
    XT[(kNB * j + c) + (int64_t)r * kb2] = v;
  }
  __syncthreads();   // orders this work-group's global stores before its own reads
  for (int i = j + 1; i < nsub; ++i) {
    const int sbi = min(kNB, kb2 - kNB * i);
    typename V4<T>::type acc[2][2];
    zero_acc<T>(acc);
    gemm_tile<T, false, true>(Lf + (k2 + kNB * i) + (int64_t)(k2 + kNB * j) * n, n,
                              X + kNB * j + (int64_t)(kNB * j) * kb2, kb2, sbi, sbj, kNB * (i - j), acc, sA, sB);
    T* Xij = X + kNB * i + (int64_t)(kNB * j) * kb2;
    for_acc<T>(acc, [&](int r, int c, T v) {
      if (r < sbi && c < sbj) Xij[r + (int64_t)c * kb2] = v;
    });
    __syncthreads();
    zero_acc<T>(acc);
    gemm_tile<T, false, true>(Dinv + S.Doff[s] + (int64_t)(blk0 + i) * kNB * kNB, kNB, Xij, kb2, sbi, sbj, sbi,
                              acc, sA, sB);
    __syncthreads();
    T* XTji = XT + kNB * j + (int64_t)(kNB * i) * kb2;
    for_acc<T>(acc, [&](int r, int c, T v) {
      if (r < sbi && c < sbj) {
        Xij[r + (int64_t)c * kb2] = -v;
        XTji[c + (int64_t)r * kb2] = -v;
      }
    });
    __syncthreads();
  }
}

// X = L[R', K] Linv_KK, stored transposed: Y[c + r * 256] holds X[r, c] (r = 0 is the
// first row of R'), so that every product reading Y takes it with its block columns
// contiguous; 128x128 tiles, Linv_KK read through its stored transpose D2T
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sel_Y2(DevSym S, LaunchList L, int step, SelBufs<T> B,
                                                     const int64_t* __restrict__ D2off, const T* __restrict__ D2T) {
  __shared__ __attribute__((aligned(16))) T sA[BigLds<T>::v];
  __shared__ __attribute__((aligned(16))) T sB[BigLds<T>::v];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const OuterBlk o = outer_blk(p, n, step);
  const int nct = (o.kb2 + kBT - 1) / kBT;
  const int rt = (int)(loc / nct), ctile = (int)(loc % nct);
  const int row0 = o.rs + kBT * rt, col0 = kBT * ctile;
  const int M = min(kBT, n - row0), N = min(kBT, o.kb2 - col0);
  const T* XT = D2T + D2off[s] + (int64_t)o.K * kNB2 * kNB2;
  typename V4<T>::type acc[4][4];
  zero_acc128<T>(acc);
  // Linv_KK is lower triangular: the columns from col0 on take only its rows from col0 on
  gemm_tile128<T, false, false>(B.L + S.Loff[s] + row0 + (int64_t)(o.k2 + col0) * n, n,
                                XT + col0 + (int64_t)col0 * o.kb2, o.kb2, M, N, o.kb2 - col0, acc, sA, sB);
  T* Y = B.Y + S.Voff[s] * kNB2;
  for_acc128<T>(acc, [&](int r, int c, T v) {
    if (r < M && c < N) Y[(col0 + c) + (int64_t)(row0 - o.rs + r) * kNB2] = v;
  });
}

// Sigma[R', K] = -Sigma[R', R'] Y, mirrored into Sigma[K, R']; 128x128 tiles
// Two waves per SIMD, for the same reason as k_update (FP64 selected inversion of the
// 1M-unknown space-time posterior: 1585 -> 1197 ms).
template <typename T>
__global__ __launch_bounds__(kThreads, 2) void k_sel_gemm2(DevSym S, LaunchList L, int step, SelBufs<T> B) {
  __shared__ __attribute__((aligned(16))) T sA[BigLds<T>::v];
  __shared__ __attribute__((aligned(16))) T sB[BigLds<T>::v];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const OuterBlk o = outer_blk(p, n, step);
  const int split = L.aux[2 * fi];
  const int nct = (o.kb2 + kBT - 1) / kBT;
  const int tile = (int)(loc / split), sp = (int)(loc % split);
  const int rt = tile / nct, ctile = tile % nct;
  const int row0 = o.rs + kBT * rt, col0 = kBT * ctile;
  const int M = min(kBT, n - row0), N = min(kBT, o.kb2 - col0);
  const int np = n - o.rs;
  const int kpart = ((np + split - 1) / split + BigTK<T>::v - 1) / BigTK<T>::v * BigTK<T>::v;
  const int kb = min(np, sp * kpart), ke = min(np, kb + kpart);
  T* Sf = B.Scur + S.Woff[s];
  const T* Y = B.Y + S.Voff[s] * kNB2;
  typename V4<T>::type acc[4][4];
  zero_acc128<T>(acc);
  gemm_tile128<T, false, false>(Sf + row0 + (int64_t)(o.rs + kb) * n, n, Y + col0 + (int64_t)kb * kNB2, kNB2, M,
                                N, ke - kb, acc, sA, sB);
  if (split == 1) {
    for_acc128<T>(acc, [&](int r, int c, T v) {
      if (r < M && c < N) {
        Sf[(row0 + r) + (int64_t)(o.k2 + col0 + c) * n] = -v;
        Sf[(o.k2 + col0 + c) + (int64_t)(row0 + r) * n] = -v;
      }
    });
  } else {
    T* out = B.gpart + wg_id() * (int64_t)(kBT * kBT);
    for_acc128<T>(acc, [&](int r, int c, T v) { out[r + c * kBT] = v; });
  }
}

// FP32 Sigma[R', K] = -Sigma[R', R'] Y in 256 x 256 tiles (the whole outer block per
// work-group), split over K like k_sel_gemm2 (partials are 256 x 256, column-major).
__global__ __launch_bounds__(kThreads4, 1) void k_sel_gemm4(DevSym S, LaunchList L, int step, SelBufs<float> B) {
  __shared__ G4Smem sm;
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const OuterBlk o = outer_blk(p, n, step);
  const int split = L.aux[2 * fi];
  const int rt = (int)(loc / split), sp = (int)(loc % split);
  const int row0 = o.rs + kG4 * rt;
  const int M = min(kG4, n - row0), N = o.kb2;
  const int np = n - o.rs;
  const int kpart = ((np + split - 1) / split + kG4K - 1) / kG4K * kG4K;
  const int kb = min(np, sp * kpart), ke = min(np, kb + kpart);
  float* Sf = B.Scur + S.Woff[s];
  const float* Y = B.Y + S.Voff[s] * kNB2;
  f16v_t acc[4][2];
  zero_acc6(acc);
  gemm_tile4(Sf + row0 + (int64_t)(o.rs + kb) * n, n, Y + (int64_t)kb * kNB2, kNB2, M, N, ke - kb, acc, sm.g);
  if (split == 1) {
    g4_epilogue<true>(acc, sm, [&](int r, int c, float v) {
      if (r < M && c < N) Sf[(row0 + r) + (int64_t)(o.k2 + c) * n] = -v;
    }, [&](int r, int c, float v) {
      if (r < M && c < N) Sf[(o.k2 + c) + (int64_t)(row0 + r) * n] = -v;
    });
  } else {
    float* out = B.gpart + wg_id() * (int64_t)(kG4 * kG4);
    g4_epilogue<false>(acc, sm, [&](int r, int c, float v) { out[r + c * kG4] = v; }, [](int, int, float) {});
  }
}

// Sum of the split-K partials of one TM x NC tile of Sigma[R', K] (128 x 128 tiles, FP32
// 256 x 256 tiles) in a fixed order, written to Sigma[R', K] and its mirror Sigma[K, R'].
// aux = (split, first work-group of the front in the partial launch).  One work-group per
// 64-column group of a tile: the sums are formed with coalesced reads, written down the
// columns, and staged in LDS so that the mirror is written along its rows.
template <typename T, int TM, int NC>
__global__ __launch_bounds__(kThreads) void k_sel_gemm_reduce(DevSym S, LaunchList L, int step, SelBufs<T> B) {
  __shared__ T tileS[64][TM + 1];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const OuterBlk o = outer_blk(p, n, step);
  const int split = L.aux[2 * fi];
  const int64_t base = L.aux[2 * fi + 1];
  constexpr int NQ = NC / 64;
  const int nct = (o.kb2 + NC - 1) / NC;
  const int tile = (int)(loc / NQ), quarter = (int)(loc % NQ);
  const int rt = tile / nct, ctile = tile % nct;
  const int row0 = o.rs + TM * rt, col0 = NC * ctile + 64 * quarter;
  const int M = min(TM, n - row0), N = min(64, o.kb2 - col0);
  if (N <= 0) return;
  constexpr int64_t PT = (int64_t)TM * NC;
  const T* pp = B.gpart + (base + (int64_t)tile * split) * PT + (int64_t)(64 * quarter) * TM;
  T* Sf = B.Scur + S.Woff[s];
  constexpr int U = 8;
  for (int e0 = threadIdx.x; e0 < TM * 64; e0 += kThreads * U) {
    T a[U];
    sum_parts<T, U>(pp, PT, split, e0, kThreads, a);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kThreads, r = e % TM, c = e / TM;
      tileS[c][r] = -a[u];
      if (r < M && c < N) Sf[(row0 + r) + (int64_t)(o.k2 + col0 + c) * n] = -a[u];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TM * 64; e += kThreads) {
    const int c = e & 63, r = e >> 6;
    if (r < M && c < N) Sf[(o.k2 + col0 + c) + (int64_t)(row0 + r) * n] = tileS[c][r];
  }
}

// split-K partials of X^T Sigma[R', K]: work-group (front, chunk, ti, tj) computes the
// 64x64 tile (ti, tj) over kSelChunk rows of R' into part + wg * 64^2; Sigma[R', K] is read
// through its stored mirror Sigma[K, R'] (rows contiguous)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sel_part2(DevSym S, LaunchList L, int step, SelBufs<T> B) {
  __shared__ T sA[kTile64Lds];
  __shared__ T sB[kTile64Lds];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const OuterBlk o = outer_blk(p, n, step);
  const int nt = o.nsub * o.nsub;
  const int chunk = (int)(loc / nt), rem = (int)(loc % nt);
  const int ti = rem / o.nsub, tj = rem % o.nsub;
  if (ti < tj) return;   // only the lower tiles of the symmetric block are read
  const int r0 = kSelChunk * chunk;
  const int kr = max(0, min(kSelChunk, n - o.rs - r0));
  const int M = min(kNB, o.kb2 - kNB * ti), N = min(kNB, o.kb2 - kNB * tj);
  const T* Sf = B.Scur + S.Woff[s];
  const T* Y = B.Y + S.Voff[s] * kNB2;
  typename V4<T>::type acc[2][2];
  zero_acc<T>(acc);
  if (kr > 0)
    gemm_tile<T, false, false>(Y + kNB * ti + (int64_t)r0 * kNB2, kNB2,
                               Sf + (o.k2 + kNB * tj) + (int64_t)(o.rs + r0) * n, n, M, N, kr, acc, sA, sB);
  T* out = B.part + wg_id() * (kNB * kNB);
  for_acc<T>(acc, [&](int r, int c, T v) { out[r + c * kNB] = v; });
}

// Sigma[K, K] tile (ti >= tj) = (Linv^T Linv)[ti, tj] - sum over chunks of the partials,
// written to both triangles
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sel_fin2(DevSym S, LaunchList L, LaunchList Lpart, int step,
                                                       SelBufs<T> B, const int64_t* __restrict__ D2off,
                                                       const T* __restrict__ D2) {
  __shared__ T sA[kTile64Lds];
  __shared__ T sB[kTile64Lds];
  int fi; int64_t loc;
  find_front(L, wg_id(), fi, loc);
  const int s = L.fronts[fi];
  const int n = fn(S, s), p = fp(S, s);
  const OuterBlk o = outer_blk(p, n, step);
  const int ti = (int)(loc / o.nsub), tj = (int)(loc % o.nsub);
  if (ti < tj) return;
  const int M = min(kNB, o.kb2 - kNB * ti), N = min(kNB, o.kb2 - kNB * tj);
  const T* X = D2 + D2off[s] + (int64_t)o.K * kNB2 * kNB2;
  typename V4<T>::type acc[2][2];
  zero_acc<T>(acc);
  // (Linv^T Linv)[ti, tj], ti >= tj: the columns of Linv in block ti are zero above row
  // 64 ti, so the sum starts there
  const int k0 = kNB * ti;
  gemm_tile<T, true, true>(X + (int64_t)(kNB * ti) * o.kb2 + k0, o.kb2, X + (int64_t)(kNB * tj) * o.kb2 + k0, o.kb2,
                           M, N, o.kb2 - k0, acc, sA, sB);
  const int nt = o.nsub * o.nsub;
  const int64_t q0 = Lpart.prefix[fi];
  const int nchunks = (int)((Lpart.prefix[fi + 1] - q0) / nt);
  T* Sf = B.Scur + S.Woff[s];
  const T* pp = B.part + (q0 + ti * o.nsub + tj) * (int64_t)(kNB * kNB);
  const int64_t pstride = (int64_t)nt * (kNB * kNB);
  for_acc<T>(acc, [&](int r, int c, T v) {
    if (r < M && c < N) {
      // fixed-order sum of the chunk partials, eight independent loads in flight
      const T* q = pp + r + c * kNB;
      T sp = T(0);
      int ch = 0;
      for (; ch + 8 <= nchunks; ch += 8) {
        T w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = q[(ch + u) * pstride];
#pragma unroll
        for (int u = 0; u < 8; ++u) sp += w[u];
      }
      for (; ch < nchunks; ++ch) sp += q[ch * pstride];
      const T val = v - sp;
      if (ti == tj && r < c) return;   // the diagonal tile writes its lower half only
      const int gi = o.k2 + kNB * ti + r, gj = o.k2 + kNB * tj + c;
      Sf[gi + (int64_t)gj * n] = val;
      Sf[gj + (int64_t)gi * n] = val;
    }
  });
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_sel_extract(DevSym S, LaunchList L, SelBufs<T> B,
                                                          const double* __restrict__ scale, double* __restrict__ var) {
  const int s = L.fronts[blockIdx.x];
  const int n = fn(S, s), p = fp(S, s);
  const T* Sf = B.Scur + S.Woff[s];
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    const int32_t o = S.perm[S.sfirst[s] + j];
    const double sc = scale[o];
    var[o] = sc * sc * (double)Sf[j + (int64_t)j * n];
  }
}

template <typename T>
__global__ void k_sel_pattern(int64_t cnt, const int64_t* __restrict__ map_e, const int64_t* __restrict__ map_off,
                              const int32_t* __restrict__ qrow, const int32_t* __restrict__ qcol,
                              const double* __restrict__ scale, const T* __restrict__ Sc,
                              double* __restrict__ sigq) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = map_e[i];
    if (e < 0) e = -e - 1;
    sigq[e] = scale[qrow[e]] * scale[qcol[e]] * (double)Sc[map_off[i]];
  }
}

inline unsigned grid_for(int64_t n, int64_t cap = 65536) {
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}


// ---- level-fused solves (one right-hand side) ----
// One launch per tree depth.  Every 64-row chunk of every front of the depth is one
// work-group task; a work-group takes the next ticket at its start (tickets follow the
// task list order, in which every task comes after the tasks it depends on), so a task
// only ever waits for tasks that already run or have finished.  The x blocks of a front
// are produced in order by its pivot chunks, and prog[s] counts the blocks published.
// Everything read inside the launch that another work-group wrote in it (x blocks and
// counters) is written and read with device-scope atomic accesses, which are coherent
// across the XCDs' L2 caches: the producer writes its block, waits for those stores to
// complete, then stores the counter; a consumer polls the counter and then loads the
// block, both at device scope.  No L2 write-back or invalidation is needed, so the other
// work-groups' cached data stays put.  A wait longer than kSpinLimit polls sets *err and
// stops waiting (the result is then wrong and the error is reported), so every launch
// terminates.
constexpr int kSpinLimit = 1 << 20;
// forward-pass groups whose fronts have at most this many rows run one task per wave
constexpr int kWaveTaskRows = 256;
// work-groups of a whole-forest pass (four per CU, more than fit at once); each takes groups
// of tasks by ticket until none is left, so that a pass over a forest of many fronts is not
// one work-group dispatch per group
constexpr int kForestGrid = 1024;

__device__ __forceinline__ double load_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll prog until it reaches `need`; returns the value seen (uniform over the
// work-group).  Two barriers: every wave has read the slot before it is reused.
__device__ __forceinline__ int wait_progress(int32_t* prog, int need, int32_t* err, int* slot) {
  if (threadIdx.x == 0) {
    int v = __hip_atomic_load(prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int spins = 0;
    while (v < need) {
      if (++spins > kSpinLimit) {
        atomicOr(err, 1);
        v = INT_MAX;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      v = __hip_atomic_load(prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    *slot = v;
  }
  __syncthreads();
  const int v = *slot;
  __syncthreads();
  return v;
}

// The block's device-scope stores are all issued by wave 0 (lanes < 64), to which
// thread 0 belongs: waiting for its outstanding memory operations orders them before
// the counter store.
__device__ __forceinline__ void publish_progress(int32_t* prog, int value) {
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_store(prog, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- whole-forest solves: one launch per pass ----
// Forward, task (front s, chunk c), rows 64c..64c+63 of the front:
//   acc(row) = sum over x blocks t < min(c, P) of L[row, block t] x_t  (P = pivot blocks);
//   pivot chunk (c < P): x_c = Linv_cc (v - acc) on its pivot rows -> xp, published; its
//   rows below p also take L[row, block c] x_c; update rows (>= p): v(row) - acc goes to
//   the front's update part, read by the parent.  Wave w takes columns 16w..16w+15 of
//   every block, lanes take rows, and the waves' sums are added in a fixed order.
// Backward, task (front s, pivot chunk c), chunks from the right: r_j = y_j - sum over the
//   rows below the block of L[row, j] x(row); x_c = Linv_cc^T r over y in xp, published as
//   prog[s] = P - c.  Wave w accumulates columns 16w..16w+15 over lanes = rows and sums its
//   lanes with a fixed butterfly.
// The tasks of every depth in one launch: the forward takes the deepest fronts first,
// the backward the roots first.  On top of the within-front x-block waits of the
// level-fused kernels, a forward task first waits until its front's children have
// written their update rows (kids[s] == need[s]) and then forms its rows of the front
// vector itself -- the right-hand side on pivot rows plus the children's entries in a
// fixed child order through the gather map -- so no separate extend-add pass is needed;
// a backward task first waits until its parent front has published all of its x blocks,
// which implies every ancestor has.  A work-group takes one ticket and runs a group of
// consecutive tasks in order (tasks of small fronts are grouped, up to 16, so that a pass
// over a forest of many small fronts needs far fewer work-groups and ticket atomics).
// Tasks only wait for tasks earlier in the list, which belong to lower tickets or come
// earlier in the same group, so the launch always progresses.
__device__ __forceinline__ int wait_count(int32_t* ctr, int need, int32_t* err, int* slot) {
  return wait_progress(ctr, need, err, slot);
}

// Wave-level forward tasks for the groups of small fronts (at most 256 rows): each wave of
// the work-group runs its own tasks of the group (tasks w, w + 4, ... in order), with lanes
// on the 64 rows of its chunk, values of other lanes broadcast by lane reads, and waits
// polled by lane 0 without work-group barriers.  (The backward pass keeps one task per
// work-group: with lanes on rows its column sums need cross-lane reductions, which the
// four waves share there.)
// Every wave still only waits for earlier tasks, and the earliest unfinished task of a
// group is always the one its wave is running, so the group progresses.
__device__ __forceinline__ int wave_wait(int32_t* ctr, int need, int32_t* err) {
  int v = 0;
  if ((threadIdx.x & 63) == 0) {
    v = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int spins = 0;
    while (v < need) {
      if (++spins > kSpinLimit) {
        atomicOr(err, 1);
        v = INT_MAX;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      v = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  return __builtin_amdgcn_readfirstlane(v);
}

// the wave's stores are complete before lane 0 stores the counter
__device__ __forceinline__ void wave_publish(int32_t* prog, int value) {
  if ((threadIdx.x & 63) == 0) {
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_store(prog, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// sum over k < kend of col(k)[lane] * v_k, v_k the value of lane k; column loads in
// batches of 16
template <typename T, typename Col>
__device__ __forceinline__ double wave_gemv(Col col, double v, int kend) {
  double acc = 0.0;
  for (int k0 = 0; k0 < kend; k0 += 16) {
    T cv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) cv[u] = col(min(k0 + u, kend - 1));
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double vk = readlane_f64(v, min(k0 + u, 63));
      acc += k0 + u < kend ? (double)cv[u] * vk : 0.0;
    }
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ void fwd_task_wave(const DevSym& S, const FusedTasks& F, const ForestBufs& G,
                                              const T* __restrict__ Lp, const T* __restrict__ D, double* xp,
                                              int s, int c) {
  const int n = fn(S, s), p = fp(S, s);
  const int P = (p + 63) >> 6;
  const int nb = min(c, P);
  const int lane = threadIdx.x & 63;
  const int row = 64 * c + lane;
  const T* Lr = Lp + S.Loff[s] + min(row, n - 1);
  const int64_t f0 = S.sfirst[s];
  int32_t* prog = F.prog + s;
  if (G.need[s] > 0) (void)wave_wait(G.kids + s, G.need[s], F.err);
  double vi = 0.0;
  if (row < n) {
    vi = row < p ? xp[f0 + row] : 0.0;
    const int64_t r0 = G.roff[s] + row;
    for (int64_t e = G.gptr[r0]; e < G.gptr[r0 + 1]; ++e) vi += load_dev(G.U + G.gsrc[e]);
  }
  double acc = 0.0;
  for (int t = 0; t < nb; ++t) {
    (void)wave_wait(prog, t + 1, F.err);
    const int q = min(64 * t + lane, p - 1);
    const double x = load_dev(xp + f0 + q);
    acc += wave_gemv<T>([&](int k) { return Lr[(int64_t)(64 * t + k) * n]; }, x, min(64, p - 64 * t));
  }
  double extra = 0.0;
  if (c < P) {
    const int pb = min(64, p - 64 * c);
    const T* Db = D + S.Doff[s] + (int64_t)c * kNB * kNB;
    const double xsrc = lane < pb ? vi - acc : 0.0;
    const double xc = wave_gemv<T>([&](int k) { return Db[lane + k * kNB]; }, xsrc, pb);
    if (lane < pb) store_dev(xp + f0 + 64 * c + lane, xc);
    wave_publish(prog, c + 1);
    if (64 * c + 64 > p && n > p)
      extra = wave_gemv<T>([&](int k) { return Lr[(int64_t)(64 * c + k) * n]; }, xc, pb);
  }
  if (64 * c + 63 >= p && n > p) {
    if (row >= p && row < n) store_dev(G.U + G.uoff[s] + (row - p), vi - acc - extra);
    const int par = G.parent[s];
    if (lane == 0 && par >= 0) {
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_fetch_add(G.kids + par, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fwd_forest(DevSym S, FusedTasks F, ForestBufs G,
                                                         const T* __restrict__ Lp, const T* __restrict__ D,
                                                         double* xp, const double* __restrict__ skip) {
  __shared__ int s_task, s_slot;
  __shared__ double red[4][64];
  __shared__ double xs[64];
  __shared__ double vin[64];
  if (skip && skip[0] == 0.0) return;
  for (;;) {
  if (threadIdx.x == 0) s_task = atomicAdd(F.ticket, 1);
  __syncthreads();
  const int grp = s_task;
  __syncthreads();   // every wave has read the ticket before thread 0 takes the next one
  if (grp >= F.count) break;
  const int t_end = F.group[grp + 1];
  if (fn(S, F.task[F.group[grp]].x) <= kWaveTaskRows) {
    for (int ti = F.group[grp] + (int)(threadIdx.x >> 6); ti < t_end; ti += kThreads / 64)
      fwd_task_wave<T>(S, F, G, Lp, D, xp, F.task[ti].x, F.task[ti].y);
    continue;
  }
  for (int ti = F.group[grp]; ti < t_end; ++ti) {
  const int2 tk = F.task[ti];
  const int s = tk.x, c = tk.y;
  const int n = fn(S, s), p = fp(S, s);
  const int P = (p + 63) >> 6;
  const int nb = min(c, P);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = 64 * c + lane;
  const T* Lr = Lp + S.Loff[s] + min(row, n - 1);
  const int64_t f0 = S.sfirst[s];
  int32_t* prog = F.prog + s;
  const bool piv = c < P;
  T dv[16];
  if (piv) {
    const T* Db = D + S.Doff[s] + (int64_t)c * kNB * kNB;
#pragma unroll
    for (int u = 0; u < 16; ++u) dv[u] = Db[lane + (16 * w + u) * kNB];
  }
  auto load_l = [&](int t, T* l) {
    const int cb = 64 * t + 16 * w;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int cc = min(cb + u, p - 1);
      l[u] = Lr[(int64_t)cc * n] * (T)(cb + u < p);
    }
  };
  T lc[16], ln[16];
  if (nb > 0) load_l(0, lc);
  // this chunk's rows of the front vector: right-hand side on pivot rows, plus the
  // children's update entries once every child chunk holding update rows has finished
  if (G.need[s] > 0) (void)wait_count(G.kids + s, G.need[s], F.err, &s_slot);
  if (w == 0) {
    double vi = 0.0;
    if (row < n) {
      vi = row < p ? xp[f0 + row] : 0.0;
      const int64_t r0 = G.roff[s] + row;
      for (int64_t e = G.gptr[r0]; e < G.gptr[r0 + 1]; ++e) vi += load_dev(G.U + G.gsrc[e]);
    }
    vin[lane] = vi;
  }
  double acc = 0.0;
  int ready = 0;
  for (int t = 0; t < nb; ++t) {
    if (t + 1 < nb) load_l(t + 1, ln);
    if (t >= ready) ready = wait_progress(prog, t + 1, F.err, &s_slot);
    const int q = min(64 * t + lane, p - 1);
    const double x = load_dev(xp + f0 + q) * (double)(64 * t + lane < p);
#pragma unroll
    for (int u = 0; u < 16; ++u) acc += (double)lc[u] * readlane_f64(x, 16 * w + u);
#pragma unroll
    for (int u = 0; u < 16; ++u) lc[u] = ln[u];
  }
  red[w][lane] = acc;
  __syncthreads();
  const double tot = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
  double extra = 0.0;
  if (piv) {
    const int pb = min(64, p - 64 * c);
    __syncthreads();
    if (w == 0) xs[lane] = lane < pb ? vin[lane] - tot : 0.0;
    __syncthreads();
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) part += (double)dv[u] * xs[16 * w + u];
    red[w][lane] = part;
    __syncthreads();
    const double xc = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    if (w == 0 && lane < pb) store_dev(xp + f0 + 64 * c + lane, xc);
    publish_progress(prog, c + 1);
    if (64 * c + 64 > p && n > p) {
      if (w == 0) xs[lane] = lane < pb ? xc : 0.0;
      __syncthreads();
      double e = 0.0;
      const int cb0 = 64 * c + 16 * w;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int cc = min(cb0 + u, p - 1);
        e += (double)(Lr[(int64_t)cc * n] * (T)(cb0 + u < p)) * xs[16 * w + u];
      }
      red[w][lane] = e;
      __syncthreads();
      extra = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    }
  }
  // update rows -> the front's update part; the chunk then counts for its parent
  if (64 * c + 63 >= p && n > p) {
    if (w == 0 && row >= p && row < n) store_dev(G.U + G.uoff[s] + (row - p), vin[lane] - tot - extra);
    const int par = G.parent[s];
    if (threadIdx.x == 0 && par >= 0) {
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_fetch_add(G.kids + par, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();   // the shared buffers are reused by the group's next task
  }
  }
}

// Sums over the 64 lanes of a wave of NV values per lane (NV = 16 or 64): a butterfly in
// which each of the first log2(NV) levels hands half of the lane's values to its partner
// and keeps the partner's half of the other values, and the remaining levels add plainly.
// Lane l ends with the total of value (l & (64 - 64 / NV)) * NV / 64, after NV - 1 +
// 6 - log2(NV) exchanges instead of 6 NV.  Every total adds the lanes in the same tree
// (partners at distance 32, 16, ..., 1), whatever NV.
template <int NV, int CNT>
struct LaneFold {
  static __device__ __forceinline__ void run(double* v, int lane) {
    constexpr int H = CNT / 2;
    constexpr int M = 32 * CNT / NV;
    const bool up = (lane & M) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double send = up ? v[i] : v[i + H];
      const double keep = up ? v[i + H] : v[i];
      v[i] = keep + __shfl_xor(send, M, 64);
    }
    LaneFold<NV, H>::run(v, lane);
  }
};
template <int NV>
struct LaneFold<NV, 1> {
  static __device__ __forceinline__ void run(double* v, int) {
#pragma unroll
    for (int m = 32 / NV; m >= 1; m >>= 1) v[0] += __shfl_xor(v[0], m, 64);
  }
};

// Backward pass; NR right-hand sides share each load of L (NR = 1, or 2 for a multi-RHS
// pass, whose last group may be partial).  Each wave holds 16 column sums per right-hand
// side and folds them across its lanes in one butterfly.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_bwd_forest(DevSym S, FusedTasks F, ForestBufs G,
                                                         const T* __restrict__ Lp, const T* __restrict__ D,
                                                         double* xp, int nrhs, int64_t ldx,
                                                         const double* __restrict__ skip) {
  constexpr int NV = 16 * NR;
  __shared__ int s_task, s_slot;
  __shared__ T Ds[kNB * (kNB + 1)];
  __shared__ double rs[NR][64];
  __shared__ double red[NR][4][64];
  if (skip && skip[0] == 0.0) return;
  for (;;) {
  if (threadIdx.x == 0) s_task = atomicAdd(F.ticket, 1);
  __syncthreads();
  const int grp = s_task;
  __syncthreads();   // every wave has read the ticket before thread 0 takes the next one
  if (grp >= F.count) break;
  const int t_end = F.group[grp + 1];
  for (int ti = F.group[grp]; ti < t_end; ++ti) {
  const int2 tk = F.task[ti];
  const int s = tk.x, c = tk.y;
  const int n = fn(S, s), p = fp(S, s);
  const int P = (p + 63) >> 6;
  const int pb = min(64, p - 64 * c);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t f0 = S.sfirst[s];
  const int32_t* rows = S.rows + S.rowptr[s];
  int32_t* prog = F.prog + s;
  {
    // the pb x pb part of the inverse diagonal block; a wave's columns are uniform, so the
    // columns past pb are not read at all
    const T* Db = D + S.Doff[s] + (int64_t)c * kNB * kNB;
#pragma unroll
    for (int k = 0; k < kNB * kNB / kThreads; ++k) {
      const int e = threadIdx.x + k * kThreads;
      const int i = e & 63, j = e >> 6;
      Ds[i + j * (kNB + 1)] = (i < pb && j < pb) ? Db[e] : (T)0;
    }
  }
  const T* Lc = Lp + S.Loff[s];
  int cols[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) cols[u] = 64 * c + min(16 * w + u, pb - 1);
  // rows below p: ancestors' unknowns, final once the parent front has published them all
  const int par = G.parent[s];
  if (par >= 0 && n > p) {
    const int Pp = (fp(S, par) + 63) >> 6;
    (void)wait_count(F.prog + par, Pp, F.err, &s_slot);
  }
  int ready = 0;
  // groups of NR right-hand sides one after the other; the block's progress is published
  // once all of them are final, so the waits of the first group cover the rest
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
  const double* xg[NR];
#pragma unroll
  for (int g = 0; g < NR; ++g) xg[g] = xp + (int64_t)min(r0 + g, nrhs - 1) * ldx;
  double acc[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) acc[u] = 0.0;
  for (int rw = p; rw < n; rw += 64) {
    const int row = rw + lane;
    const int rc = min(row, n - 1);
    T lv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) lv[u] = Lc[rc + (int64_t)cols[u] * n];
    const int xi = rows[rc];
    const double m = (double)(row < n);
#pragma unroll
    for (int g = 0; g < NR; ++g) {
      const double xv = load_dev(xg[g] + xi) * m;
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[16 * g + u] += (double)lv[u] * xv;
    }
  }
  for (int t = P - 1; t > c; --t) {
    const int row = 64 * t + lane;
    const int rc = min(row, p - 1);
    T lv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) lv[u] = Lc[rc + (int64_t)cols[u] * n];
    if (ready < P - t) ready = wait_progress(prog, P - t, F.err, &s_slot);
    const double m = (double)(row < p);
#pragma unroll
    for (int g = 0; g < NR; ++g) {
      const double xv = load_dev(xg[g] + f0 + rc) * m;
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[16 * g + u] += (double)lv[u] * xv;
    }
  }
  LaneFold<NV, NV>::run(acc, lane);
  {
    const int idx = (lane & (64 - 64 / NV)) * NV / 64;   // right-hand side idx / 16, column idx % 16
    const int g = idx >> 4, jj = 16 * w + (idx & 15);
    if ((lane & (64 / NV - 1)) == 0) rs[g][jj] = jj < pb ? xg[g][f0 + 64 * c + jj] - acc[0] : 0.0;
  }
  __syncthreads();
  double part[NR];
#pragma unroll
  for (int g = 0; g < NR; ++g) part[g] = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int i = 16 * w + u;
    const double d = (double)Ds[i + lane * (kNB + 1)];
#pragma unroll
    for (int g = 0; g < NR; ++g) part[g] += d * rs[g][i];
  }
#pragma unroll
  for (int g = 0; g < NR; ++g) red[g][w][lane] = part[g];
  __syncthreads();
  if (w == 0 && lane < pb) {
#pragma unroll
    for (int g = 0; g < NR; ++g)
      if (r0 + g < nrhs)
        store_dev(xp + (int64_t)(r0 + g) * ldx + f0 + 64 * c + lane,
                  (red[g][0][lane] + red[g][1][lane]) + (red[g][2][lane] + red[g][3][lane]));
  }
  __syncthreads();   // rs and red are reused by the next group of right-hand sides
  }
  publish_progress(prog, P - c);
  __syncthreads();   // the shared buffers are reused by the group's next task
  }
  }
}

}  // namespace

// ------------------------------------------------------------------ launch wrappers
void launch_assemble_qpost(hipStream_t st, int64_t nnzq, const double* qval, const int64_t* cptr,
                           const int32_t* cpair, const int32_t* arow, const double* aval,
                           const double* qeps, double* qpost) {
  hipLaunchKernelGGL(k_assemble_qpost, dim3(grid_for(nnzq)), dim3(kThreads), 0, st, nnzq, qval, cptr,
                     cpair, arow, aval, qeps, qpost);
}
void launch_assemble_dqpost(hipStream_t st, int64_t nnzq, const double* dq, const int64_t* cptr,
                            const int32_t* cpair, const int32_t* arow, const double* aval, const double* da,
                            const double* qeps, const double* dqeps, double* out) {
  hipLaunchKernelGGL(k_assemble_dqpost, dim3(grid_for(nnzq)), dim3(kThreads), 0, st, nnzq, dq, cptr, cpair, arow,
                     aval, da, qeps, dqeps, out);
}
void launch_spmv_obs(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* v,
                     const double* x, double* y) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_spmv_obs, dim3(grid_for(m)), dim3(kThreads), 0, st, m, arp, aci, v, x,
                     (const double*)nullptr, (const double*)nullptr, 1, y);
}
void launch_obs_resid_plain(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* v,
                            const double* y, const double* b, const double* x, double* r) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_spmv_obs, dim3(grid_for(m)), dim3(kThreads), 0, st, m, arp, aci, v, x, y, b, 0, r);
}
void launch_elementwise(hipStream_t st, int64_t n, int mode, const double* a, const double* b, double* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_elementwise, dim3(grid_for(n)), dim3(kThreads), 0, st, n, mode, a, b, out);
}
void launch_cg_xr(hipStream_t st, int64_t n, const double* sc, const double* p, const double* q, double* x,
                  double* r) {
  hipLaunchKernelGGL(k_cg_xr, dim3(grid_for(n)), dim3(kThreads), 0, st, n, sc, p, q, x, r);
}
void launch_cg_p(hipStream_t st, int64_t n, double* sc, const double* z, double* p) {
  hipLaunchKernelGGL(k_cg_p, dim3(grid_for(n)), dim3(kThreads), 0, st, n, sc, z, p);
  hipLaunchKernelGGL(k_cg_roll, dim3(1), dim3(64), 0, st, sc);
}
void launch_copy_f64(hipStream_t st, int64_t n, const double* a, double* b) {
  hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(n)), dim3(kThreads), 0, st, n, a, b);
}
void launch_jacobi(hipStream_t st, int64_t n, const int64_t* qdiag, const double* qv, const double* r, double* z) {
  hipLaunchKernelGGL(k_jacobi, dim3(grid_for(n)), dim3(kThreads), 0, st, n, qdiag, qv, r, z);
}
void launch_rbmc(hipStream_t st, int64_t n, const int64_t* rp, const int32_t* ci, const double* qv,
                 const int64_t* qdiag, int64_t k, const double* xs, double* var) {
  hipLaunchKernelGGL(k_rbmc, dim3(grid_for(n)), dim3(kThreads), 0, st, n, rp, ci, qv, qdiag, k, xs, var);
}
void launch_obs_residual(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci,
                         const double* aval, const double* qeps, const double* y, const double* b,
                         const double* mu, double* rvec) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_obs_residual, dim3(grid_for(m)), dim3(kThreads), 0, st, m, arp, aci, aval, qeps,
                     y, b, mu, rvec);
}
void launch_at_times(hipStream_t st, int64_t n, const int64_t* atp, const int32_t* ati,
                     const int32_t* arow, const double* aval, const double* rvec, double* h) {
  hipLaunchKernelGGL(k_at_times, dim3(grid_for(n)), dim3(kThreads), 0, st, n, atp, ati, arow, aval, rvec, h);
}
void launch_equilibrate(hipStream_t st, int64_t n, int64_t nnzq, const int64_t* qdiag,
                        const int32_t* qrow, const int32_t* qcol, const double* qpost, int32_t* sexp,
                        double* scale, double* qhat) {
  hipLaunchKernelGGL(k_equil_rows, dim3(grid_for(n)), dim3(kThreads), 0, st, n, qdiag, qpost, sexp, scale);
  hipLaunchKernelGGL(k_equil_vals, dim3(grid_for(nnzq)), dim3(kThreads), 0, st, nnzq, qdiag, qrow, qcol,
                     qpost, qhat);
}
void launch_fill_i32(hipStream_t st, int32_t* p, int64_t n, int32_t v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n)), dim3(kThreads), 0, st, p, n, v);
}
void launch_fill_f64(hipStream_t st, double* p, int64_t n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n)), dim3(kThreads), 0, st, p, n, v);
}

template <typename T> void launch_zero_lower(hipStream_t st, const DevSym& S, const LaunchList& L, T* W) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_zero_lower<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, W);
}
template <typename T> void launch_scatter(hipStream_t st, int64_t cnt, const int64_t* map_e,
                                          const int64_t* map_off, const double* qhat, T* W) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_scatter<T>, dim3(grid_for(cnt)), dim3(kThreads), 0, st, cnt, map_e, map_off, qhat, W);
}
template <typename T> void launch_extend_add(hipStream_t st, const DevSym& S, const LaunchList& L, int slot,
                                             const T* Wchild, T* Wcur) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_extend_add<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, slot, Wchild, Wcur);
}
template <typename T> void launch_potrf(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                        NumBufs<T> B) {
  if (L.count <= 0) return;
  hipLaunchKernelGGL(k_potrf<T>, dim3((unsigned)L.count), dim3(kThreads), 0, st, S, L, step, B);
}
template <typename T> void launch_trsm(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                       NumBufs<T> B) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_trsm<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, step, B);
}
template <typename T> void launch_update(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                         int mode, NumBufs<T> B) {
  if (L.total <= 0) return;
  if (mode == 0)
    hipLaunchKernelGGL((k_update<T, 64>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, step, mode, B);
  else
    hipLaunchKernelGGL((k_update<T, 128>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, step, mode, B);
}
template <typename T> void launch_copy_L(hipStream_t st, const DevSym& S, const LaunchList& L, NumBufs<T> B) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_copy_L<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, B);
}
void launch_logdet(hipStream_t st, int64_t nblocks, const int64_t* bptr, const int32_t* bpiv,
                   const int32_t* perm, const double* piv, const int32_t* sexp, double* part, double* out) {
  hipLaunchKernelGGL(k_logdet, dim3((unsigned)(nblocks * kLdParts)), dim3(kThreads), 0, st, bptr, bpiv, perm, piv,
                     sexp, part);
  hipLaunchKernelGGL(k_logdet_final, dim3((unsigned)((nblocks + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                     nblocks, (const double*)part, out);
}

template <typename T> void launch_fvec_init(hipStream_t st, const DevSym& S, const LaunchList& L, SolveBufs V) {
  if (L.count <= 0) return;
  hipLaunchKernelGGL(k_fvec_init<T>, dim3((unsigned)L.count), dim3(kThreads), 0, st, S, L, V);
}
template <typename T> void launch_fvec_extend(hipStream_t st, const DevSym& S, const LaunchList& L, int slot,
                                              SolveBufs V) {
  if (L.count <= 0) return;
  hipLaunchKernelGGL(k_fvec_extend<T>, dim3((unsigned)L.count), dim3(kThreads), 0, st, S, L, slot, V);
}
template <typename T> void launch_fwd_block(hipStream_t st, const DevSym& S, const LaunchList& L, int t,
                                            const T* D2, const int64_t* D2off, SolveBufs V) {
  if (L.total <= 0) return;
  if (V.nrhs == 1)
    hipLaunchKernelGGL((k_fwd_block<T, 1>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, t, D2, D2off, V);
  else
    hipLaunchKernelGGL((k_fwd_block<T, 16>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, t, D2, D2off, V);
}
template <typename T> void launch_inv256(hipStream_t st, const DevSym& S, const LaunchList& L, const T* Lbase,
                                         int from_front, const T* Dinv, const int64_t* D2off, T* D2, T* D2T) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_inv256<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, Lbase, from_front, Dinv,
                     D2off, D2, D2T);
}
template <typename T> void launch_fwd_outer(hipStream_t st, const DevSym& S, const LaunchList& L, int t,
                                            const T* Lp, SolveBufs V) {
  if (L.total <= 0) return;
  if (V.nrhs == 1)
    hipLaunchKernelGGL((k_fwd_outer<T, 1>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, t, Lp, V);
  else
    hipLaunchKernelGGL((k_fwd_outer<T, 16>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, t, Lp, V);
}
template <typename T> void launch_bwd_part(hipStream_t st, const DevSym& S, const LaunchList& L, int t,
                                           const T* Lp, SolveBufs V, double* part) {
  if (L.total <= 0) return;
  if (V.nrhs == 1)
    hipLaunchKernelGGL((k_bwd_part<T, 1>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, t, Lp, V, part);
  else
    hipLaunchKernelGGL((k_bwd_part<T, 16>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, t, Lp, V, part);
}
template <typename T> void launch_bwd_block(hipStream_t st, const DevSym& S, const LaunchList& L,
                                            const LaunchList& Lpart, int t, const T* D2T, const int64_t* D2off,
                                            SolveBufs V, const double* part) {
  if (L.total <= 0) return;
  if (V.nrhs == 1)
    hipLaunchKernelGGL((k_bwd_block<T, 1>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, Lpart, t, D2T,
                       D2off, V, part);
  else
    hipLaunchKernelGGL((k_bwd_block<T, 16>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, Lpart, t, D2T,
                       D2off, V, part);
}

template <typename T> void launch_fwd_forest(hipStream_t st, const DevSym& S, FusedTasks F, ForestBufs G,
                                             const T* Lp, const T* D, double* xp, const double* skip) {
  if (F.count <= 0) return;
  hipLaunchKernelGGL(k_fwd_forest<T>, dim3((unsigned)min(F.count, kForestGrid)), dim3(kThreads), 0, st, S, F, G,
                     Lp, D, xp, skip);
}
template <typename T> void launch_bwd_forest(hipStream_t st, const DevSym& S, FusedTasks F, ForestBufs G,
                                             const T* Lp, const T* D, double* xp, int nrhs, int64_t ldx,
                                             const double* skip) {
  if (F.count <= 0) return;
  if (nrhs > 1)
    hipLaunchKernelGGL((k_bwd_forest<T, 2>), dim3((unsigned)min(F.count, kForestGrid)), dim3(kThreads), 0, st, S,
                       F, G, Lp, D, xp, nrhs, ldx, skip);
  else
    hipLaunchKernelGGL((k_bwd_forest<T, 1>), dim3((unsigned)min(F.count, kForestGrid)), dim3(kThreads), 0, st, S,
                       F, G, Lp, D, xp, nrhs, ldx, skip);
}
void launch_permute_in(hipStream_t st, int64_t n, int nrhs, const int32_t* perm, const double* scale,
                       const double* src, int64_t lds, double* xp, const double* gate) {
  hipLaunchKernelGGL(k_permute_in, dim3(grid_for(n * nrhs)), dim3(kThreads), 0, st, n, nrhs, perm, scale, src,
                     lds, xp, gate);
}
void launch_refine_gate(hipStream_t st, const double* norms, double tol, double* gate, double* rec, int record) {
  hipLaunchKernelGGL(k_refine_gate, dim3(1), dim3(64), 0, st, norms, tol, gate, rec, record);
}
void launch_permute_in_f32(hipStream_t st, int64_t n, int nrhs, const float* z, double* xp) {
  hipLaunchKernelGGL(k_permute_in_f32, dim3(grid_for(n * nrhs)), dim3(kThreads), 0, st, n * nrhs, z, xp);
}
void launch_permute_out(hipStream_t st, int64_t n, int nrhs, const int32_t* perm, const double* scale,
                        const double* xp, const double* add, int64_t ldadd, double* out, int64_t ldo,
                        int accumulate) {
  hipLaunchKernelGGL(k_permute_out, dim3(grid_for(n * nrhs)), dim3(kThreads), 0, st, n, nrhs, perm, scale, xp,
                     add, ldadd, out, ldo, accumulate);
}
void launch_resid(hipStream_t st, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                  const double* h, const double* x, double* r) {
  hipLaunchKernelGGL(k_resid, dim3(grid_for(n * kRowG)), dim3(kThreads), 0, st, n, rp, ci, val, h, x, r);
}
void launch_matern_values(hipStream_t st, int64_t nnz, const double* mv, const double* sv, const double* smsv,
                          double kappa, double tau, double* q, double* dq) {
  hipLaunchKernelGGL(k_matern_values, dim3(grid_for(nnz)), dim3(kThreads), 0, st, nnz, mv, sv, smsv, kappa, tau,
                     q, dq);
}
void launch_spmv(hipStream_t st, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                 const double* x, double* y) {
  hipLaunchKernelGGL(k_spmv, dim3(grid_for(n * kRowG)), dim3(kThreads), 0, st, n, rp, ci, val, x, y);
}
void launch_weighted_resid(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* aval,
                           const double* qeps, const double* y, const double* b, const double* x, double* w) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_weighted_resid, dim3(grid_for(m)), dim3(kThreads), 0, st, m, arp, aci, aval, qeps, y, b, x, w);
}
void launch_burgers_linearize(hipStream_t st, int64_t nx, int64_t nt, double dt, double nu, const double* mass,
                              const double* s3, const double* u, const int64_t* arp, double* aval, double* b) {
  hipLaunchKernelGGL(k_burgers_linearize, dim3(grid_for(nx * nt)), dim3(kThreads), 0, st, nx, nt, dt, nu, mass, s3, u,
                     arp, aval, b);
}
void launch_gn_linesearch(hipStream_t st, int64_t nx, int64_t nt, double dt, double nu, const double* mass,
                          const double* s3, const double* u, const double* d, const double* y, const double* qeps,
                          const int64_t* arp, const int32_t* aci, const double* aval, double* part,
                          const double* quad, double* sel, double* rec) {
  hipLaunchKernelGGL(k_burgers_trials, dim3(kRedBlocksGN), dim3(256), 0, st, nx, nt, dt, nu, mass, s3, u, d, y, qeps,
                     arp, aci, aval, part);
  hipLaunchKernelGGL(k_gn_select, dim3(1), dim3(64), 0, st, (const double*)part, quad, sel, rec);
}
void launch_pw_linearize(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* lin,
                         const int32_t* nl_col, const double* nl_coef, int power, const double* u, double* aval,
                         double* b) {
  hipLaunchKernelGGL(k_pw_linearize, dim3(grid_for(m)), dim3(kThreads), 0, st, m, arp, aci, lin, nl_col, nl_coef,
                     power, u, aval, b);
}
void launch_pw_linesearch(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* lin,
                          const int32_t* nl_col, const double* nl_coef, int power, const double* u, const double* d,
                          const double* y, const double* qeps, const double* aval, double* part, const double* quad,
                          double* sel, double* rec) {
  hipLaunchKernelGGL(k_pw_trials, dim3(kRedBlocksGN), dim3(256), 0, st, m, arp, aci, lin, nl_col, nl_coef, power, u,
                     d, y, qeps, aval, part);
  hipLaunchKernelGGL(k_gn_select, dim3(1), dim3(64), 0, st, (const double*)part, quad, sel, rec);
}
void launch_gn_direction(hipStream_t st, int64_t n, const double* x, const double* u, double* d) {
  hipLaunchKernelGGL(k_gn_direction, dim3(grid_for(n)), dim3(kThreads), 0, st, n, x, u, d);
}
void launch_gn_update(hipStream_t st, int64_t n, const double* sel, const double* d, double* u) {
  hipLaunchKernelGGL(k_gn_update, dim3(grid_for(n)), dim3(kThreads), 0, st, n, sel, d, u);
}
void launch_add(hipStream_t st, int64_t n, const double* a, const double* b, double* out) {
  hipLaunchKernelGGL(k_add, dim3(grid_for(n)), dim3(kThreads), 0, st, n, a, b, out);
}
void launch_norm2(hipStream_t st, int64_t n, const double* v, double* partial, double* out) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(kThreads), 0, st, n, v, (const double*)nullptr, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kThreads), 0, st, partial, 1, out);
}
void launch_dot(hipStream_t st, int64_t n, const double* a, const double* b, double* partial, double* out) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(kThreads), 0, st, n, a, b, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kThreads), 0, st, partial, 0, out);
}

template <typename T> void launch_sel_gather(hipStream_t st, const DevSym& S, const LaunchList& L,
                                             const int32_t* sparent, SelBufs<T> B) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_sel_gather<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, sparent, B);
}
template <typename T> void launch_sel_Y2(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                         SelBufs<T> B, const int64_t* D2off, const T* D2) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_sel_Y2<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, step, B, D2off, D2);
}
template <typename T> void launch_sel_gemm2(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                            SelBufs<T> B) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_sel_gemm2<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, step, B);
}
template <typename T> void launch_sel_gemm_reduce(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                                  SelBufs<T> B) {
  if (L.total <= 0) return;
  if constexpr (std::is_same<T, float>::value)
    hipLaunchKernelGGL((k_sel_gemm_reduce<float, kG4, kG4>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L,
                       step, B);
  else
    hipLaunchKernelGGL((k_sel_gemm_reduce<T, 128, 128>), dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, step,
                       B);
}
void launch_cg_iteration(hipStream_t st, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                         const int64_t* qdiag, double* sc, int cur, double* x, double* r, double* z, double* p,
                         double* q, double* part) {
  double* part_pq = part;
  double* part_rz = part + kCgBlocks;
  double* part_rr = part + 2 * kCgBlocks;
  hipLaunchKernelGGL(k_cg_spmv_pq, dim3(kCgBlocks), dim3(kThreads), 0, st, n, rp, ci, val, (const double*)p, q,
                     part_pq);
  hipLaunchKernelGGL(k_cg_sum, dim3(1), dim3(kThreads), 0, st, (const double*)part_pq, sc + 2);
  hipLaunchKernelGGL(k_cg_update, dim3(kCgBlocks), dim3(kThreads), 0, st, n, (const double*)sc, cur,
                     (const double*)p, (const double*)q, x, r, qdiag, val, z, part_rz, part_rr);
  hipLaunchKernelGGL(k_cg_sum, dim3(1), dim3(kThreads), 0, st, (const double*)part_rz, sc + (1 - cur));
  hipLaunchKernelGGL(k_cg_pupdate, dim3(kCgBlocks), dim3(kThreads), 0, st, n, (const double*)sc, cur,
                     (const double*)z, p);
}
void launch_partial_norm(hipStream_t st, const double* part, double* out) {
  hipLaunchKernelGGL(k_cg_sum, dim3(1), dim3(kThreads), 0, st, part + 2 * kCgBlocks, out + 2);
  hipLaunchKernelGGL(k_cg_sqrt, dim3(1), dim3(1), 0, st, out);
}
void launch_sel_gemm4(hipStream_t st, const DevSym& S, const LaunchList& L, int step, SelBufs<float> B) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_sel_gemm4, dim3((unsigned)L.total), dim3(kThreads4), 0, st, S, L, step, B);
}
void launch_panel_upd4(hipStream_t st, const DevSym& S, const LaunchList& L, int K, NumBufs<float> B, float* part) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_panel_upd4, dim3((unsigned)L.total), dim3(kThreads4), 0, st, S, L, K, B, part);
}
void launch_panel_red4(hipStream_t st, const DevSym& S, const LaunchList& L, int K, NumBufs<float> B,
                       const float* part) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_panel_red4, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, K, B, part);
}
void launch_syrk4(hipStream_t st, const DevSym& S, const LaunchList& L, NumBufs<float> B) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_syrk4, dim3((unsigned)L.total), dim3(kThreads4), 0, st, S, L, B);
}
template <typename T> void launch_sel_part2(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                            SelBufs<T> B) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_sel_part2<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, step, B);
}
template <typename T> void launch_sel_fin2(hipStream_t st, const DevSym& S, const LaunchList& L,
                                           const LaunchList& Lpart, int step, SelBufs<T> B,
                                           const int64_t* D2off, const T* D2) {
  if (L.total <= 0) return;
  hipLaunchKernelGGL(k_sel_fin2<T>, dim3((unsigned)L.total), dim3(kThreads), 0, st, S, L, Lpart, step, B, D2off, D2);
}
template <typename T> void launch_sel_extract(hipStream_t st, const DevSym& S, const LaunchList& L, SelBufs<T> B,
                                              const double* scale, double* var) {
  if (L.count <= 0) return;
  hipLaunchKernelGGL(k_sel_extract<T>, dim3((unsigned)L.count), dim3(kThreads), 0, st, S, L, B, scale, var);
}
template <typename T> void launch_sel_pattern(hipStream_t st, int64_t cnt, const int64_t* map_e,
                                              const int64_t* map_off, const int32_t* qrow, const int32_t* qcol,
                                              const double* scale, const T* Scur, double* sigq) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_sel_pattern<T>, dim3(grid_for(cnt)), dim3(kThreads), 0, st, cnt, map_e, map_off, qrow, qcol,
                     scale, Scur, sigq);
}


#define GMRF_INST(T)                                                                                  \
  template void launch_zero_lower<T>(hipStream_t, const DevSym&, const LaunchList&, T*);            \
  template void launch_scatter<T>(hipStream_t, int64_t, const int64_t*, const int64_t*, const double*, T*); \
  template void launch_extend_add<T>(hipStream_t, const DevSym&, const LaunchList&, int, const T*, T*); \
  template void launch_potrf<T>(hipStream_t, const DevSym&, const LaunchList&, int, NumBufs<T>);     \
  template void launch_trsm<T>(hipStream_t, const DevSym&, const LaunchList&, int, NumBufs<T>);      \
  template void launch_update<T>(hipStream_t, const DevSym&, const LaunchList&, int, int, NumBufs<T>); \
  template void launch_copy_L<T>(hipStream_t, const DevSym&, const LaunchList&, NumBufs<T>);         \
  template void launch_fvec_init<T>(hipStream_t, const DevSym&, const LaunchList&, SolveBufs);       \
  template void launch_fvec_extend<T>(hipStream_t, const DevSym&, const LaunchList&, int, SolveBufs); \
  template void launch_fwd_block<T>(hipStream_t, const DevSym&, const LaunchList&, int, const T*, const int64_t*, SolveBufs); \
  template void launch_fwd_outer<T>(hipStream_t, const DevSym&, const LaunchList&, int, const T*, SolveBufs); \
  template void launch_bwd_part<T>(hipStream_t, const DevSym&, const LaunchList&, int, const T*, SolveBufs, double*); \
  template void launch_bwd_block<T>(hipStream_t, const DevSym&, const LaunchList&, const LaunchList&, int, const T*, const int64_t*, SolveBufs, const double*); \
  template void launch_fwd_forest<T>(hipStream_t, const DevSym&, FusedTasks, ForestBufs, const T*, const T*, double*, const double*); \
  template void launch_bwd_forest<T>(hipStream_t, const DevSym&, FusedTasks, ForestBufs, const T*, const T*, double*, int, int64_t, const double*); \
  template void launch_sel_gather<T>(hipStream_t, const DevSym&, const LaunchList&, const int32_t*, SelBufs<T>); \
  template void launch_inv256<T>(hipStream_t, const DevSym&, const LaunchList&, const T*, int, const T*, const int64_t*, T*, T*); \
  template void launch_sel_Y2<T>(hipStream_t, const DevSym&, const LaunchList&, int, SelBufs<T>, const int64_t*, const T*); \
  template void launch_sel_gemm2<T>(hipStream_t, const DevSym&, const LaunchList&, int, SelBufs<T>); \
  template void launch_sel_gemm_reduce<T>(hipStream_t, const DevSym&, const LaunchList&, int, SelBufs<T>); \
  template void launch_sel_part2<T>(hipStream_t, const DevSym&, const LaunchList&, int, SelBufs<T>); \
  template void launch_sel_fin2<T>(hipStream_t, const DevSym&, const LaunchList&, const LaunchList&, int, SelBufs<T>, const int64_t*, const T*); \
  template void launch_sel_extract<T>(hipStream_t, const DevSym&, const LaunchList&, SelBufs<T>, const double*, double*); \
  template void launch_sel_pattern<T>(hipStream_t, int64_t, const int64_t*, const int64_t*, const int32_t*, const int32_t*, const double*, const T*, double*);
GMRF_INST(double)
GMRF_INST(float)
#undef GMRF_INST

}  // namespace gmrf
