// Device kernels of the symmetric-TensorMap library, written for CDNA4
// (gfx950, 64-wide wavefronts, MFMA, 160 KiB LDS per CU).
//
//  * permute_kernel: Alg. "Abelian Tensor Permutation" executed as a list of
//    block tasks (one fusion channel, or a chunk of one); also writes the
//    zero blocks of coupled charges with an empty K range.
//  * gemm_f64_kernel: persistent grouped GEMM over the coupled charges of a
//    contraction (eq. abelian_compostion), fp64 MFMA 16x16x4; its epilogue
//    applies the output permute of Alg. "Abelian tensor contraction" by
//    scattering every element straight to its place in C.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "tk_internal.h"

namespace tk {

// Device memory pointers in the global address space: pointers read from
// the buffer table would otherwise be generic (flat) pointers, whose loads
// count against the LDS wait counter and serialise with LDS traffic.
#define TK_GLOBAL __attribute__((address_space(1)))
// read-only tables (tiles, GEMM descriptors) read through the constant
// address space: uniform loads from it become scalar loads even in kernels
// that store to global memory
#ifdef __HIP_DEVICE_COMPILE__
#define TK_CONST __attribute__((address_space(4)))
#else
#define TK_CONST
#endif
template <typename T>
__device__ __forceinline__ const TK_CONST T* const_ptr(const T* p) {
  return (const TK_CONST T*)p;
}

template <typename T>
__device__ __forceinline__ TK_GLOBAL T* buf_ptr(const Ptrs& P, int id) {
  return (TK_GLOBAL T*)(P.table ? reinterpret_cast<void*>(const_ptr(P.table)[id]) : P.p[id]);
}

// ---------------------------------------------------------------------------
// permute / zero-fill
// ---------------------------------------------------------------------------
// Each thread handles up to kBatch elements of a task at a time: all their
// offsets and loads are issued before any store, so many loads are in flight
// per thread (the kernel is bound by HBM bandwidth and latency, not ALU).
constexpr int kBatch = 8;

// One element as a split-BF16x3 operand: hi = bf16(x) (x rounded to fp32
// first), lo = bf16(x - hi); hi + lo keeps about 16 significant bits.
template <typename T>
__device__ __forceinline__ void store_split(TK_GLOBAL __bf16* hi, int64_t lo, T v) {
  const float x = static_cast<float>(v);
  const __bf16 h = static_cast<__bf16>(x);
  hi[0] = h;
  hi[lo] = static_cast<__bf16>(x - static_cast<float>(h));
}

// A task's source and destination buffer ids (adjacent 16-bit fields, the
// first 4-byte aligned) as one 32-bit scalar load: a 16-bit field read on its
// own compiles to a vector load, whose round trip would delay the task's
// first data loads.
template <typename TaskT>
__device__ __forceinline__ void load_buf_ids(const TaskT* __restrict__ tk, int* src_buf, int* dst_buf) {
  static_assert(__builtin_offsetof(TaskT, src_buf) % 4 == 0 &&
                    __builtin_offsetof(TaskT, dst_buf) == __builtin_offsetof(TaskT, src_buf) + 2,
                "adjacent 16-bit buffer ids");
  const uint32_t w = __builtin_amdgcn_readfirstlane(*reinterpret_cast<const uint32_t*>(&tk->src_buf));
  *src_buf = static_cast<int16_t>(w & 0xffffu);
  *dst_buf = static_cast<int16_t>(w >> 16);
}

// A task's divisions by its dimensions (extent, multiply-high magic and
// shift per dimension), read once as wave-uniform values (scalar registers):
// the eight 1-byte shift counts as one 8-byte word, since a byte array read
// at every use compiles to a vector byte load per lane.  The task record is
// the same for every thread that calls this (a workgroup's or a wave's).
template <typename TaskT>
__device__ __forceinline__ void load_divisors(const TaskT* __restrict__ tk, int32_t* dim, uint32_t* mag,
                                              uint32_t* shr) {
  static_assert(__builtin_offsetof(TaskT, shr) % 8 == 0, "8-byte aligned shift counts");
  const uint64_t shr8 = *reinterpret_cast<const uint64_t*>(tk->shr);
#pragma unroll
  for (int d = 0; d < kMaxDims; ++d) {
    dim[d] = __builtin_amdgcn_readfirstlane(tk->dim[d]);
    mag[d] = __builtin_amdgcn_readfirstlane(tk->mag[d]);
    shr[d] = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(shr8 >> (8 * d)) & 0xffu);
  }
}

// One task, processed by `nthr` threads starting at thread `t0` of the
// workgroup (the whole workgroup for a large task, one wave for small ones).
// SPLIT: tasks with lo != 0 write bf16 hi and lo planes instead of T.
// The task record is uniform over those threads (scalar loads), and element
// offsets are 32-bit, relative to the task's source and destination: a
// block holds fewer than 2^31 elements (the planner refuses larger ones) and
// a split plane fewer than 2^31 values.
template <typename T, bool SPLIT = false>
__device__ __forceinline__ void permute_task(const PermTask* __restrict__ tk, const Ptrs& P, double alpha,
                                             double beta, int lt, int nthr) {
  const int n = tk->n;
  const int count = tk->count;
  const uint32_t start = static_cast<uint32_t>(tk->start);
  const T sign = static_cast<T>(tk->sign);
  int32_t dim[kMaxDims], ss[kMaxDims], ds[kMaxDims];
  uint32_t mag[kMaxDims], shr[kMaxDims];
  load_divisors(tk, dim, mag, shr);
#pragma unroll
  for (int d = 0; d < kMaxDims; ++d) {
    ss[d] = __builtin_amdgcn_readfirstlane(tk->ss[d]);
    ds[d] = __builtin_amdgcn_readfirstlane(tk->ds[d]);
  }
  int sbuf, dbuf;
  load_buf_ids(tk, &sbuf, &dbuf);
  TK_GLOBAL T* __restrict__ dst = buf_ptr<T>(P, dbuf) + tk->dst;
  const bool has_src = sbuf >= 0;
  const TK_GLOBAL T* __restrict__ src = buf_ptr<const T>(P, has_src ? sbuf : dbuf) + tk->src;
  for (int e0 = 0; e0 < count; e0 += nthr * kBatch) {
    int32_t so[kBatch], dof[kBatch];
    T v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      // out-of-range lanes repeat the last element (loads stay in bounds and
      // unconditional; their stores are skipped)
      const int e = min(e0 + u * nthr + lt, count - 1);
      uint32_t lin = start + static_cast<uint32_t>(e);
      int32_t a = 0, b = 0;
#pragma unroll
      for (int d = 0; d < kMaxDims; ++d) {
        if (d < n) {
          // lin < 2^31: division by dim[d] as a multiply-high (host-side magic)
          const uint32_t q = static_cast<uint32_t>((static_cast<uint64_t>(lin) * mag[d]) >> shr[d]);
          const uint32_t i = lin - q * static_cast<uint32_t>(dim[d]);
          lin = q;
          a += static_cast<int32_t>(i) * ss[d];
          b += static_cast<int32_t>(i) * ds[d];
        }
      }
      so[u] = a;
      dof[u] = b;
    }
    if (has_src) {
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = src[so[u]] * sign;
    } else {
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = static_cast<T>(0);
    }
    if (beta != 0.0) {
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int e = e0 + u * nthr + lt;
        if (e < count) v[u] = static_cast<T>(alpha) * v[u] + static_cast<T>(beta) * dst[dof[u]];
      }
    } else if (alpha != 1.0) {
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = static_cast<T>(alpha) * v[u];
    }
    if (SPLIT && tk->lo != 0) {
      // the operand permute of a split-BF16x3 plan (alpha 1, beta 0)
      TK_GLOBAL __bf16* hi = (TK_GLOBAL __bf16*)buf_ptr<void>(P, dbuf) + tk->dst;
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int e = e0 + u * nthr + lt;
        if (e < count) store_split(hi + dof[u], tk->lo, v[u]);
      }
      continue;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * nthr + lt;
      if (e < count) dst[dof[u]] = v[u];
    }
  }
}

// A workgroup holding one task spreads it over all its threads; one holding
// several small tasks gives each wave its own tasks, so their loads are in
// flight together instead of one task after another.
template <typename T, bool SPLIT = false>
__global__ __launch_bounds__(kThreads) void permute_kernel(const PermTask* __restrict__ tasks,
                                                           const int32_t* __restrict__ wg_first,
                                                           Ptrs P, double alpha, double beta) {
  const int t0 = wg_first[blockIdx.x];
  const int t1 = wg_first[blockIdx.x + 1];
  if (t1 - t0 == 1) {
    permute_task<T, SPLIT>(tasks + t0, P, alpha, beta, threadIdx.x, kThreads);
    return;
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int t = t0 + wave; t < t1; t += kThreads / 64) permute_task<T, SPLIT>(tasks + t, P, alpha, beta, lane, 64);
}

// Block permute through LDS, one tile per workgroup: the tile is read with
// consecutive lanes along the source's contiguous dimension a (16 rows of
// 64 lanes per pass, all loads of a thread issued before the first LDS
// store), staged as [ib][ia] with a padded row, and written with consecutive
// lanes along the destination's contiguous dimension b.  Used where a block's
// source and destination are contiguous along different dimensions (a plain
// output-order walk would gather its reads or scatter its writes).
template <typename T, bool SPLIT>
__global__ __launch_bounds__(kThreads) void permute_tile_kernel(const TileTask* __restrict__ tiles, Ptrs P,
                                                                double alpha, double beta) {
  constexpr int E = kTileEdge, R = kThreads / E;  // R rows per pass
  __shared__ T tile[E][E + 1];
  const TileTask tk = tiles[blockIdx.x];
  const int lane = threadIdx.x % E, row = threadIdx.x / E;
  const T sign = static_cast<T>(tk.sign);
  const bool has_src = tk.src_buf >= 0;
  if (has_src) {
    const TK_GLOBAL T* __restrict__ src = buf_ptr<const T>(P, tk.src_buf) + tk.src;
    T v[E / R];
#pragma unroll
    for (int u = 0; u < E / R; ++u) {
      const int ib = row + R * u;
      v[u] = (lane < tk.ea && ib < tk.eb) ? src[lane + static_cast<int64_t>(ib) * tk.sb] : static_cast<T>(0);
    }
#pragma unroll
    for (int u = 0; u < E / R; ++u) tile[row + R * u][lane] = v[u] * sign;
  }
  __syncthreads();
  // write: lane runs along b, rows along a
#pragma unroll 4
  for (int ia = row; ia < tk.ea; ia += R) {
    if (lane >= tk.eb) continue;
    const T x = has_src ? tile[lane][ia] : static_cast<T>(0);
    const int64_t o = static_cast<int64_t>(ia) * tk.ta + lane;
    if (SPLIT && tk.lo != 0) {
      store_split((TK_GLOBAL __bf16*)buf_ptr<void>(P, tk.dst_buf) + tk.dst + o, tk.lo, x);
      continue;
    }
    TK_GLOBAL T* __restrict__ dst = buf_ptr<T>(P, tk.dst_buf) + tk.dst;
    T y = static_cast<T>(alpha) * x;
    if (beta != 0.0) y += static_cast<T>(beta) * dst[o];
    dst[o] = y;
  }
}

// Partial trace: each thread takes kTraceUnroll output elements at once;
// their indices in the block are split over the output dimensions once, then
// each contribution adds coef * (sum along its traced diagonal) -- the
// diagonal walk is the same for every element of a task, so each of its
// steps issues the loads of all the thread's elements before adding them
// (a walk per element would wait one memory latency per diagonal entry) --
// and each element is written once (alpha times the trace plus beta times
// the old value).  Lanes past the task's end repeat its last element (loads
// stay in bounds) and skip the store.
constexpr int kTraceUnroll = 4;

template <typename T>
__device__ __forceinline__ void trace_task(const TraceTask* __restrict__ tk, const TraceContrib* __restrict__ cs,
                                           const Ptrs& P, double alpha, double beta, int lt, int nthr) {
  constexpr int U = kTraceUnroll;
  const int n = tk->n, count = tk->count, c0 = tk->c0, c1 = tk->c1;
  const uint32_t start = static_cast<uint32_t>(tk->start);
  int sbuf, dbuf;
  load_buf_ids(tk, &sbuf, &dbuf);
  TK_GLOBAL T* __restrict__ dst = buf_ptr<T>(P, dbuf) + tk->dst;
  const TK_GLOBAL T* __restrict__ src = buf_ptr<const T>(P, sbuf);
  int32_t dim[kMaxDims];
  uint32_t mag[kMaxDims], shr[kMaxDims];
  load_divisors(tk, dim, mag, shr);
  for (int e0 = lt; e0 < count; e0 += U * nthr) {
    int32_t idx[U][kMaxDims];
    int64_t dof[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t lin = start + static_cast<uint32_t>(min(e0 + u * nthr, count - 1));
      dof[u] = 0;
#pragma unroll
      for (int d = 0; d < kMaxDims; ++d) {
        idx[u][d] = 0;
        if (d < n) {
          const uint32_t q = static_cast<uint32_t>((static_cast<uint64_t>(lin) * mag[d]) >> shr[d]);
          const uint32_t i = lin - q * static_cast<uint32_t>(dim[d]);
          lin = q;
          idx[u][d] = static_cast<int32_t>(i);
          dof[u] += static_cast<int64_t>(i) * tk->ds[d];
        }
      }
    }
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    for (int c = c0; c < c1; ++c) {
      const TraceContrib* cb = cs + c;
      int64_t base[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        base[u] = cb->src;
#pragma unroll
        for (int d = 0; d < kMaxDims; ++d)
          if (d < n) base[u] += static_cast<int64_t>(idx[u][d]) * cb->ss[d];
      }
      const int nd = cb->nd;
      int32_t t[kMaxTracePairs] = {0, 0, 0, 0};
      double sum[U];
#pragma unroll
      for (int u = 0; u < U; ++u) sum[u] = 0.0;
      for (;;) {  // every diagonal index of the traced pairs, first pair fastest
        int64_t o = 0;
#pragma unroll
        for (int j = 0; j < kMaxTracePairs; ++j)
          if (j < nd) o += static_cast<int64_t>(t[j]) * cb->dstr[j];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = static_cast<double>(src[base[u] + o]);
#pragma unroll
        for (int u = 0; u < U; ++u) sum[u] += v[u];
        int j = 0;
        for (; j < nd; ++j) {
          if (++t[j] < cb->dd[j]) break;
          t[j] = 0;
        }
        if (j == nd) break;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc[u] += cb->coef * sum[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e0 + u * nthr >= count) break;
      double v = alpha * acc[u];
      if (beta != 0.0) v += beta * static_cast<double>(dst[dof[u]]);
      dst[dof[u]] = static_cast<T>(v);
    }
  }
}

// The same task when no contribution has a traced pair and all of a task's
// contributions share their strides (the inputs of one output array differ
// only in where they start, as in a recoupling): per element the source
// offset is formed once, and each thread takes kGatherUnroll elements at
// once so that all of their loads (every element times every term) are in
// flight together.
constexpr int kGatherUnroll = 8;

template <typename T>
__device__ __forceinline__ void gather_task(const TraceTask* __restrict__ tk, const TraceContrib* __restrict__ cs,
                                            const Ptrs& P, double alpha, double beta, int lt, int nthr) {
  const int n = tk->n, count = tk->count, c0 = tk->c0, c1 = tk->c1;
  const uint32_t start = static_cast<uint32_t>(tk->start);
  int sbuf, dbuf;
  load_buf_ids(tk, &sbuf, &dbuf);
  TK_GLOBAL T* __restrict__ dst = buf_ptr<T>(P, dbuf) + tk->dst;
  const TK_GLOBAL T* __restrict__ src = buf_ptr<const T>(P, sbuf);
  int32_t ss[kMaxDims] = {0, 0, 0, 0, 0, 0, 0, 0};  // the shared source strides (none without terms)
  if (c1 > c0) {
#pragma unroll
    for (int d = 0; d < kMaxDims; ++d) ss[d] = cs[c0].ss[d];
  }
  int32_t dim[kMaxDims];
  uint32_t mag[kMaxDims], shr[kMaxDims];
  load_divisors(tk, dim, mag, shr);
  for (int e0 = lt; e0 < count; e0 += kGatherUnroll * nthr) {
    int64_t dof[kGatherUnroll], rel[kGatherUnroll];
    double acc[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const int e = e0 + u * nthr;
      uint32_t lin = start + static_cast<uint32_t>(e < count ? e : 0);
      dof[u] = 0;
      rel[u] = 0;
      acc[u] = 0.0;
#pragma unroll
      for (int d = 0; d < kMaxDims; ++d) {
        if (d < n) {
          const uint32_t q = static_cast<uint32_t>((static_cast<uint64_t>(lin) * mag[d]) >> shr[d]);
          const int64_t i = static_cast<int64_t>(lin - q * static_cast<uint32_t>(dim[d]));
          lin = q;
          dof[u] += i * tk->ds[d];
          rel[u] += i * ss[d];
        }
      }
    }
    for (int c = c0; c < c1; ++c) {
      const int64_t base = cs[c].src;
      const double coef = cs[c].coef;
      double v[kGatherUnroll];
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u)
        v[u] = e0 + u * nthr < count ? static_cast<double>(src[base + rel[u]]) : 0.0;
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) acc[u] += coef * v[u];
    }
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      if (e0 + u * nthr >= count) break;
      double r = alpha * acc[u];
      if (beta != 0.0) r += beta * static_cast<double>(dst[dof[u]]);
      dst[dof[u]] = static_cast<T>(r);
    }
  }
}

template <typename T, bool GATHER>
__global__ __launch_bounds__(kThreads) void trace_kernel(const TraceTask* __restrict__ tasks,
                                                         const int32_t* __restrict__ wg_first,
                                                         const TraceContrib* __restrict__ cs, Ptrs P, double alpha,
                                                         double beta) {
  const int t0 = wg_first[blockIdx.x];
  const int t1 = wg_first[blockIdx.x + 1];
  if (t1 - t0 == 1) {
    if (GATHER)
      gather_task<T>(tasks + t0, cs, P, alpha, beta, threadIdx.x, kThreads);
    else
      trace_task<T>(tasks + t0, cs, P, alpha, beta, threadIdx.x, kThreads);
    return;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = t0 + wave; t < t1; t += kThreads / 64) {
    if (GATHER)
      gather_task<T>(tasks + t, cs, P, alpha, beta, lane, 64);
    else
      trace_task<T>(tasks + t, cs, P, alpha, beta, lane, 64);
  }
}

typedef double d4_t __attribute__((ext_vector_type(4)));

// One-sided (Hestenes) Jacobi SVD of the coupled-sector matrices, as a
// block method spread over the whole GPU.  Each sector matrix (m x n, the
// taller side as rows) is copied into W, with V = I.  Its columns form
// blocks of kSvdBlock; a sweep pairs every two blocks once, in rounds of
// disjoint block pairs (round-robin order), and every pair of every sector
// in a round is one workgroup.  The workgroup forms the Gram matrix
// G = W_K^T W_K of its k <= 2 kSvdBlock columns, and unless all of them are
// already orthogonal (to eps max(4, sqrt(m))), applies one cyclic Jacobi sweep to G (each
// column pair rotated, by the same rotation the one-sided method would
// apply to W, in k - 1 rounds of disjoint pairs), accumulating the
// rotations in J; then W_K <- W_K J and V_K <- V_K J.  The host runs sweeps
// until one rotates nothing in a sector (a sector that rotated nothing in a
// sweep is skipped from then on: its columns no longer change).  Last, each
// column's norm is its singular value and W's columns are normalised (U).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__global__ __launch_bounds__(kSvdThreads) void svd_init_kernel(const SvdSector* __restrict__ secs,
                                                               const double* __restrict__ X,
                                                               double* __restrict__ ws) {
  const SvdSector sc = secs[blockIdx.x];
  const int m = sc.m, n = sc.n, R = sc.R;
  double* W = ws + sc.w;
  double* V = ws + sc.v;
  const double* Xs = X + sc.x;
  for (int64_t e = threadIdx.x; e < static_cast<int64_t>(m) * n; e += kSvdThreads) {
    const int i = static_cast<int>(e % m), j = static_cast<int>(e / m);
    W[e] = sc.trans ? Xs[j + static_cast<int64_t>(R) * i] : Xs[i + static_cast<int64_t>(R) * j];
  }
  for (int64_t e = threadIdx.x; e < static_cast<int64_t>(n) * n; e += kSvdThreads)
    V[e] = (e % n == e / n) ? 1.0 : 0.0;
}

// Rows of W_K (or V_K) staged in LDS per pass.
constexpr int kSvdRows = 64;
// Inner Jacobi sweeps over a block pair's Gram matrix at most (more inner
// sweeps barely reduce the outer ones: one is the cheapest overall).
constexpr int kSvdInner = 1;

// One block pair (see above); `prev` holds each sector's rotation flag of
// the previous sweep (skip the sector when it is 0), `flag` this sweep's.
// The Gram matrix and the products W_K J, V_K J run on the fp64 MFMA
// (16x16x4: lane l supplies X[l%16][l/16] and Y[l/16][l%16], and value v of
// its result is D[l/16 + 4v][l%16] of D = X Y), one 16x16 tile per wave;
// the rows pass through LDS kSvdRows at a time, the next pass's loads in
// flight while the current one is multiplied.
__global__ __launch_bounds__(kSvdRoundThreads) void svd_round_kernel(const SvdItem* __restrict__ items,
                                                                     const SvdSector* __restrict__ secs,
                                                                     double* __restrict__ ws,
                                                                     const int32_t* __restrict__ prev,
                                                                     int32_t* __restrict__ flag, int sweep,
                                                                     double tol) {
  constexpr int KM = 2 * kSvdBlock, NT = kSvdRoundThreads, PASS = kSvdRows * KM / NT;
  static_assert(NT == (KM / 2) * 16, "one 16-thread group per column pair of a round");
  static_assert(KM == 32 && NT == 256, "four waves, one 16x16 Gram tile each");
  __shared__ double G[KM][KM + 1];
  __shared__ double J[KM][KM + 1];
  __shared__ double Wc[kSvdRows][KM + 1];
  const SvdItem it = items[blockIdx.x];
  if (sweep > 0 && prev[it.sec] == 0) return;
  const SvdSector sc = secs[it.sec];
  const int k = it.np + it.nq, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, l16 = lane & 15, g4 = lane >> 4;
  // orthogonality threshold of the sector: eps max(4, sqrt(m)) (tol = eps);
  // the rounding of an m-term inner product is of order sqrt(m) eps
  tol *= fmax(4.0, sqrt(static_cast<double>(sc.m)));
  // column c of the pair's k columns: its column of W (and of V)
  auto col = [&](int c) { return c < it.np ? it.p0 + c : it.q0 + (c - it.np); };
  double* W = ws + sc.w;
  double* V = ws + sc.v;
  // element x of a pass: row x % kSvdRows, column x / kSvdRows (coalesced
  // along each column)
  double stage[PASS];
  auto load_pass = [&](const double* X, int rows, int r0) {
#pragma unroll
    for (int e = 0; e < PASS; ++e) {
      const int x = tid + NT * e, rr = x % kSvdRows, c = x / kSvdRows;
      stage[e] = (r0 + rr < rows && c < k) ? X[r0 + rr + static_cast<int64_t>(rows) * col(c)] : 0.0;
    }
  };
  auto store_pass = [&]() {
#pragma unroll
    for (int e = 0; e < PASS; ++e) {
      const int x = tid + NT * e;
      Wc[x % kSvdRows][x / kSvdRows] = stage[e];
    }
  };

  // 1. Gram matrix: wave w forms tile (w / 2, w % 2)
  const int ti = wave >> 1, tj = wave & 1;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  load_pass(W, sc.m, 0);
  for (int r0 = 0; r0 < sc.m; r0 += kSvdRows) {
    store_pass();
    __syncthreads();
    if (r0 + kSvdRows < sc.m) load_pass(W, sc.m, r0 + kSvdRows);
#pragma unroll
    for (int st = 0; st < kSvdRows / 4; ++st)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wc[4 * st + g4][16 * ti + l16], Wc[4 * st + g4][16 * tj + l16],
                                                 acc, 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) G[16 * ti + g4 + 4 * v][16 * tj + l16] = acc[v];
  for (int x = tid; x < KM * KM; x += NT) J[x / KM][x % KM] = (x / KM == x % KM) ? 1.0 : 0.0;
  __syncthreads();
  // 2. are all pairs orthogonal to tol already?
  bool rot = false;
  for (int x = tid; x < KM * KM; x += NT) {
    const int a = x / KM, b = x % KM;
    if (a < b && b < k) {
      const double ga = G[a][a], gb = G[b][b], g = G[a][b];
      rot |= ga > 0.0 && gb > 0.0 && fabs(g) > tol * sqrt(ga * gb);
    }
  }
  if (!__syncthreads_or(rot)) return;
  // 3. cyclic sweeps over the k columns until one rotates nothing (k' = k
  // rounded up to even, the extra index a dummy): round r pairs (0, 1 + r)
  // and (1 + (r + i) % (k' - 1), 1 + (r - i) % (k' - 1)), i = 1 .. k'/2 - 1
  const int kk = k + (k & 1);
  const int pi = tid / 16, p16 = tid % 16;
  for (int inner = 0; inner < kSvdInner; ++inner) {
    bool any = false;
    for (int r = 0; r < kk - 1; ++r) {
      const int p = pi == 0 ? 0 : 1 + (r + pi) % (kk - 1);
      const int q = pi == 0 ? 1 + r : 1 + (r - pi + kk - 1) % (kk - 1);
      bool doit = 2 * pi < kk && p < k && q < k;
      double c = 1.0, s = 0.0;
      if (doit) {
        const double a = G[p][p], b = G[q][q], g = G[p][q];
        doit = a > 0.0 && b > 0.0 && fabs(g) > tol * sqrt(a * b);
        if (doit) {
          const double zeta = (b - a) / (2.0 * g);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + t * t);
          s = c * t;
        }
      }
      any |= doit;
      __syncthreads();  // every rotation of the round is formed from the same G
      if (doit) {       // rows p and q: G <- R^T G
        for (int jj = p16; jj < k; jj += 16) {
          const double x = G[p][jj], y = G[q][jj];
          G[p][jj] = c * x - s * y;
          G[q][jj] = s * x + c * y;
        }
      }
      __syncthreads();
      if (doit) {  // columns p and q: G <- G R, J <- J R
        for (int ii = p16; ii < k; ii += 16) {
          const double x = G[ii][p], y = G[ii][q];
          G[ii][p] = c * x - s * y;
          G[ii][q] = s * x + c * y;
          const double u = J[ii][p], v = J[ii][q];
          J[ii][p] = c * u - s * v;
          J[ii][q] = s * u + c * v;
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(any)) break;
  }
  // 4. W_K <- W_K J and V_K <- V_K J: in each pass wave w forms rows
  // 16 w .. 16 w + 15 of the pass, both 16-column tiles
  for (int side = 0; side < 2; ++side) {
    double* X = side == 0 ? W : V;
    const int rows = side == 0 ? sc.m : sc.n;
    load_pass(X, rows, 0);
    for (int r0 = 0; r0 < rows; r0 += kSvdRows) {
      store_pass();
      __syncthreads();
      if (r0 + kSvdRows < rows) load_pass(X, rows, r0 + kSvdRows);
      d4_t o0 = {0.0, 0.0, 0.0, 0.0}, o1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < KM / 4; ++st) {
        const double a = Wc[16 * wave + l16][4 * st + g4];
        o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, J[4 * st + g4][l16], o0, 0, 0, 0);
        o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, J[4 * st + g4][16 + l16], o1, 0, 0, 0);
      }
      __syncthreads();  // the pass is read; the next store_pass may overwrite it
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 16 * wave + g4 + 4 * v;
        if (row >= rows) continue;
        if (l16 < k) X[row + static_cast<int64_t>(rows) * col(l16)] = o0[v];
        if (16 + l16 < k) X[row + static_cast<int64_t>(rows) * col(16 + l16)] = o1[v];
      }
    }
  }
  if (tid == 0) flag[it.sec] = 1;
}

// Singular values (column norms of W) and U (W's columns normalised).
__global__ __launch_bounds__(kSvdThreads) void svd_finish_kernel(const SvdSector* __restrict__ secs,
                                                                 double* __restrict__ ws) {
  const SvdSector sc = secs[blockIdx.x];
  const int m = sc.m, n = sc.n;
  double* W = ws + sc.w;
  double* S = ws + sc.s;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = kSvdThreads / 64;
  for (int j = wave; j < n; j += nw) {
    double* Wj = W + static_cast<int64_t>(m) * j;
    double a = 0.0;
    for (int i = lane; i < m; i += 64) a += Wj[i] * Wj[i];
    const double nrm = sqrt(wave_sum(a));
    if (lane == 0) S[j] = nrm;
    if (nrm > 0.0)
      for (int i = lane; i < m; i += 64) Wj[i] /= nrm;
  }
}

// Buffer id -> base address with a per-lane id (a select chain over the
// plan's buffers, or the batch's table).
template <typename T>
__device__ __forceinline__ TK_GLOBAL T* buf_ptr_lane(const Ptrs& P, int id) {
  if (P.table) return (TK_GLOBAL T*)reinterpret_cast<void*>(P.table[id]);
  void* p = P.p[0];
#pragma unroll
  for (int i = 1; i < kBufsPerPlan; ++i) p = id == i ? P.p[i] : p;
  return (TK_GLOBAL T*)p;
}

// Index map of a workgroup's chunk of concatenated ranges (elements c0 ..
// c0 + n - 1, n <= CHUNK; range i of the staged ones starts at relative
// element s_r[i], range 0 at or before the chunk): s_idx[e] = the staged
// range holding element c0 + e.  Each range marks its first element, then a
// running maximum over the chunk (per thread over CHUNK / kThreads
// consecutive entries, across the workgroup by shuffles and LDS) fills the
// rest, since later ranges have larger indices.
template <int CHUNK, typename IX>
__device__ __forceinline__ void chunk_range_map(IX* s_idx, uint32_t* s_wmax, const int32_t* s_r, int nr, int n) {
  constexpr int E = CHUNK / kThreads;
  constexpr int PER = 16 / sizeof(IX);  // entries per 16-byte word
  constexpr int BITS = 8 * sizeof(IX);
  static_assert(E * kThreads == CHUNK && E % PER == 0, "chunk size");
  uint4* s4 = reinterpret_cast<uint4*>(s_idx);
  for (int e = threadIdx.x; e < CHUNK / PER; e += kThreads) s4[e] = make_uint4(0, 0, 0, 0);
  __syncthreads();
  for (int i = 1 + threadIdx.x; i < nr; i += kThreads) {
    const int p = s_r[i];
    if (p > 0 && p < n) s_idx[p] = static_cast<IX>(i);
  }
  __syncthreads();
  uint32_t loc[E];
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < E / PER; ++q) {
    const uint4 w = s4[threadIdx.x * (E / PER) + q];
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int h = 0; h < PER; ++h) {
      m = max(m, (ws[h / (PER / 4)] >> (BITS * (h % (PER / 4)))) & ((1u << BITS) - 1u));
      loc[q * PER + h] = m;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = m;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x = max(x, y);
  }
  if (lane == 63) s_wmax[wave] = x;
  uint32_t ex = __shfl_up(x, 1, 64);
  if (lane == 0) ex = 0;
  __syncthreads();
  for (int w = 0; w < wave; ++w) ex = max(ex, s_wmax[w]);
#pragma unroll
  for (int q = 0; q < E / PER; ++q) {
    uint32_t ws[4] = {0, 0, 0, 0};
#pragma unroll
    for (int h = 0; h < PER; ++h) ws[h / (PER / 4)] |= max(ex, loc[q * PER + h]) << (BITS * (h % (PER / 4)));
    s4[threadIdx.x * (E / PER) + q] = make_uint4(ws[0], ws[1], ws[2], ws[3]);
  }
  __syncthreads();
}

// Zero ranges: workgroup w covers virtual elements wstart[w] ..
// wstart[w+1]-1 of the concatenated ranges (at most kZeroChunk elements in
// at most kZeroMax ranges).  Its ranges are staged in LDS as destination
// pointers (minus the chunk-relative start); an index map gives each
// element its range, so consecutive threads write consecutive addresses
// however short the ranges are.
template <typename T>
__global__ __launch_bounds__(kThreads) void zero_ranges_kernel(const ZeroRange* __restrict__ ranges, int nranges,
                                                               const int32_t* __restrict__ first,
                                                               const int64_t* __restrict__ wstart, Ptrs P,
                                                               double beta) {
  __shared__ TK_GLOBAL T* s_p[kZeroMax + 1];
  __shared__ int32_t s_r[kZeroMax + 1];
  __shared__ __align__(16) uint16_t s_idx[kZeroChunk];
  __shared__ uint32_t s_wmax[kThreads / 64];
  const int64_t c0 = const_ptr(wstart)[blockIdx.x], c1 = const_ptr(wstart)[blockIdx.x + 1];
  const int n = static_cast<int>(c1 - c0);
  const int r0 = const_ptr(first)[blockIdx.x];
  const int r1 = min(nranges, const_ptr(first)[blockIdx.x + 1] + 1);
  const int nr = min(r1 - r0, kZeroMax + 1);
  for (int i = threadIdx.x; i < nr; i += kThreads) {
    const ZeroRange zr = ranges[r0 + i];
    const int64_t rel = zr.vstart - c0;  // <= 0 for range 0, in (0, n] for the others
    s_r[i] = static_cast<int32_t>(max<int64_t>(rel, 0));
    s_p[i] = buf_ptr_lane<T>(P, zr.buf) + (zr.off - rel);
  }
  __syncthreads();
  if (nr > 1) chunk_range_map<kZeroChunk, uint16_t>(s_idx, s_wmax, s_r, nr, n);
  for (int e = threadIdx.x; e < n; e += kThreads) {
    TK_GLOBAL T* d = s_p[nr > 1 ? s_idx[e] : 0] + e;
    *d = beta != 0.0 ? static_cast<T>(beta) * *d : static_cast<T>(0);
  }
}

// ---------------------------------------------------------------------------
// grouped sector GEMM, fp64 MFMA
// ---------------------------------------------------------------------------

// Epilogue store of one accumulated element of C~ (row r, column s of the
// sector GEMM d): in place (mode 0) or scattered into C (mode 1).
template <typename TC>
__device__ __forceinline__ void store_elem(const GemmArgs& args, const GemmDesc& d, TK_GLOBAL TC* Cbase, int r,
                                           int s, double acc) {
  if (r >= d.M || s >= d.N) return;
  int64_t idx;
  double scale = args.alpha;
  if (d.mode == 0) {
    idx = d.c + static_cast<int64_t>(s) * d.ldc + r;
  } else {
    const LegMap rm = args.row_map[d.row_map + r];
    const LegMap cm = args.col_map[d.col_map + s];
    const PairDesc& pd = args.pairs[d.pair_base + static_cast<int64_t>(rm.chan) * d.ncc + cm.chan];
    idx = pd.base;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      idx += static_cast<int64_t>(rm.idx[l]) * pd.S[l] + static_cast<int64_t>(cm.idx[l]) * pd.S[4 + l];
    }
    scale *= pd.sign;
  }
  double v = scale * acc;
  if (args.beta != 0.0) v += args.beta * static_cast<double>(Cbase[idx]);
  Cbase[idx] = static_cast<TC>(v);
}

// MFMA of one 16x16x4 step for the arithmetic type: accumulator type, the
// call (first operand = B, so the result is the transposed tile), and where
// value v of lane l sits: column GS (l/16) + VS v of the transposed tile.
template <typename CT>
struct MfmaOf;
template <>
struct MfmaOf<double> {
  using acc = d4_t;
  static constexpr int gs = 1, vs = 4;
  static __device__ __forceinline__ d4_t mma(double b, double a, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c, 0, 0, 0);
  }
};
typedef float f4_t __attribute__((ext_vector_type(4)));
template <>
struct MfmaOf<float> {
  using acc = f4_t;
  static constexpr int gs = 4, vs = 1;
  static __device__ __forceinline__ f4_t mma(float b, float a, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c, 0, 0, 0);
  }
};

// One element through a raw buffer resource (reads zero past its records).
template <typename TS>
__device__ __forceinline__ TS buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Epilogue of a tile held transposed: value v of acc[mi][ni] is
// C[r0 + 16 mi][c0 + 16 ni + VS v] (r0, c0 already include the lane's row
// and column); the wave's sub-tile spans rows rb .. rb + 16 TM - 1 and
// columns cb .. cb + 16 TN - 1 (wave-uniform, before clipping to M x N).
// Scatter outputs (mode 1): rows (columns) of a sector are numbered channel
// by channel, so when the first and last valid row of the sub-tile share a
// channel every row does, and likewise for columns.  Then one channel pair
// covers the sub-tile: its placement is read once, through scalar loads, and
// an element's offset is a row part (once per row) plus a column part (once
// per column).  A sub-tile across channel boundaries looks up the pair of
// every element.
template <typename TS, typename AT, int TM, int TN, int VS>
__device__ __forceinline__ void store_tile_t(const GemmArgs& args, const GemmDesc& d, TK_GLOBAL TS* __restrict__ C,
                                             int r0, int c0, int rb, int cb, const AT (&acc)[TM][TN]) {
  const double alpha = args.alpha, beta = args.beta;
  if (rb >= d.M || cb >= d.N) return;  // the whole sub-tile lies outside the sector
  if (d.mode == 0) {
#pragma unroll
    for (int ni = 0; ni < TN; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = c0 + 16 * ni + VS * v;
        if (c >= d.N) continue;
#pragma unroll
        for (int mi = 0; mi < TM; ++mi) {
          const int r = r0 + 16 * mi;
          if (r >= d.M) continue;
          const int64_t x = d.c + static_cast<int64_t>(c) * d.ldc + r;
          double val = alpha * static_cast<double>(acc[mi][ni][v]);
          if (beta != 0.0) val += beta * static_cast<double>(C[x]);
          C[x] = static_cast<TS>(val);
        }
      }
    return;
  }
  const LegMap* __restrict__ rmap = args.row_map + d.row_map;
  const LegMap* __restrict__ cmap = args.col_map + d.col_map;
  const PairDesc* __restrict__ pairs = args.pairs + d.pair_base;
  LegMap rm[TM];
#pragma unroll
  for (int mi = 0; mi < TM; ++mi) rm[mi] = rmap[min(r0 + 16 * mi, d.M - 1)];
  const int rl = min(rb + 16 * TM, d.M) - 1, cl = min(cb + 16 * TN, d.N) - 1;
  const TK_CONST LegMap* rmu = const_ptr(rmap);
  const TK_CONST LegMap* cmu = const_ptr(cmap);
  const int rc = rmu[rb].chan, cc = cmu[cb].chan;
  if (rc == rmu[rl].chan && cc == cmu[cl].chan) {
    const TK_CONST PairDesc* pu = const_ptr(pairs) + static_cast<int64_t>(rc) * d.ncc + cc;
    const double scale = alpha * pu->sign;
    int32_t S[8];
#pragma unroll
    for (int l = 0; l < 8; ++l) S[l] = pu->S[l];
    int64_t R[TM];
#pragma unroll
    for (int mi = 0; mi < TM; ++mi) {
      R[mi] = pu->base;
#pragma unroll
      for (int l = 0; l < 4; ++l) R[mi] += static_cast<int64_t>(rm[mi].idx[l]) * S[l];
    }
    // The leg indices of the lane's columns (four packed 16-bit fields) are
    // loaded a group of HG column bands at a time, before that group's
    // stores: a load issued after a store waits for the store too (one
    // in-order counter).  All bands at once where the registers allow.
    constexpr int HG = TM * TN <= 4 ? TN : 1;
#pragma unroll
    for (int n0 = 0; n0 < TN; n0 += HG) {
      uint64_t cidx[HG][4];
#pragma unroll
      for (int h = 0; h < HG; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          cidx[h][v] = *reinterpret_cast<const uint64_t*>(cmap[min(c0 + 16 * (n0 + h) + VS * v, d.N - 1)].idx);
#pragma unroll
      for (int h = 0; h < HG; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ni = n0 + h;
          const int c = c0 + 16 * ni + VS * v;
          if (c >= d.N) continue;
          int64_t col = 0;
#pragma unroll
          for (int l = 0; l < 4; ++l)
            col += static_cast<int64_t>(static_cast<uint32_t>(cidx[h][v] >> (16 * l)) & 0xffffu) * S[4 + l];
#pragma unroll
          for (int mi = 0; mi < TM; ++mi) {
            if (r0 + 16 * mi >= d.M) continue;
            const int64_t x = R[mi] + col;
            double val = scale * static_cast<double>(acc[mi][ni][v]);
            if (beta != 0.0) val += beta * static_cast<double>(C[x]);
            C[x] = static_cast<TS>(val);
          }
        }
    }
    return;
  }
#pragma unroll
  for (int ni = 0; ni < TN; ++ni)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + 16 * ni + VS * v;
      if (c >= d.N) continue;
      const LegMap cm = cmap[c];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi) {
        if (r0 + 16 * mi >= d.M) continue;
        const PairDesc& pd = pairs[static_cast<int64_t>(rm[mi].chan) * d.ncc + cm.chan];
        int64_t x = pd.base;
#pragma unroll
        for (int l = 0; l < 4; ++l)
          x += static_cast<int64_t>(rm[mi].idx[l]) * pd.S[l] + static_cast<int64_t>(cm.idx[l]) * pd.S[4 + l];
        double val = alpha * pd.sign * static_cast<double>(acc[mi][ni][v]);
        if (beta != 0.0) val += beta * static_cast<double>(C[x]);
        C[x] = static_cast<TS>(val);
      }
    }
}

// Grouped sector GEMM, fp64 MFMA 16x16x4.  A workgroup of WGM x WGN waves
// owns a BM x BN tile; each wave a (BM/WGM) x (BN/WGN) sub-tile made of 16 x 16
// MFMA tiles.  K advances in stages of 16 through a double-buffered LDS tile:
// A as [k][m] (m contiguous, as in HBM), B as [n][k] (k contiguous, as in
// HBM), so every global load is coalesced along the contiguous axis.  Stage
// s+2 is fetched into registers while stage s is multiplied and is written to
// the free LDS buffer at the start of stage s+1: one barrier per stage.
// Within one MFMA the k index is lane/16; step j of the BK/4 steps of a
// stage uses k = (BK/4)*(lane/16) + j for both operands.
template <int BM, int BN, int WGM_, int WGN_, int BK_ = 16>
struct F64Tile {
  static constexpr int WGM = WGM_, WGN = WGN_;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int BK = BK_, APAD = 2, BPAD = 2;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static constexpr int A_TPM = NT / BM;  // threads sharing one m row
  static constexpr int A_LD = BK / A_TPM;
  static constexpr int B_CPL = NT / 16;  // columns of B covered per load
  static constexpr int B_LD = BN / B_CPL;
  static constexpr int NACC = TM * TN * 4;  // accumulator doubles per lane
  static_assert(NT % BM == 0 && BK % A_TPM == 0 && A_LD >= 1, "A tile");
  static_assert(BN % B_CPL == 0 && B_LD >= 1, "B tile");
  static_assert(BK % 16 == 0, "stage depth");
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile");
};


// Origin of wave w's sub-tile.  Waves w and w + NW/2 share a SIMD (waves of
// a workgroup are spread round robin over the 4 SIMDs of a CU); the first
// half of the waves covers the top row band, the second half the bottom row
// band with the column bands rotated by half, so that when the bottom rows
// or the right columns of an edge tile are empty every SIMD keeps one busy
// wave and the tile takes about half the time.
template <class TT>
__device__ __forceinline__ void wave_origin(int w, int* wm, int* wn) {
  constexpr int NW = TT::NT / 64;
  if (TT::WGM == 2 && NW >= 4) {
    const int half = NW / 2;
    const int r = w / half, c = w % half;
    *wm = r * TT::WM;
    *wn = ((c + r * (half / 2)) % half) * TT::WN;
  } else {
    *wm = (w % TT::WGM) * TT::WM;
    *wn = (w / TT::WGM) * TT::WN;
  }
}

#ifndef TK_F64_PREFETCH
#define TK_F64_PREFETCH 2
#endif

// third word of a raw buffer resource on gfx9 (32-bit data format, no
// swizzle, no stride)
constexpr int kBufWord3 = 0x00020000;

// waves per SIMD the register budget is sized for: four workgroups per CU
// for the 64 x 64 x 16 tile (128 VGPRs), two waves per SIMD otherwise
template <int BM, int BN, int BK>
constexpr int kF64WavesPerEu = (BM * BN <= 64 * 64 && BK == 16) ? 4 : 2;

// TS: element type in HBM (double or float); CT: arithmetic of the MFMAs
// (double: fp64 16x16x4, or float: fp32 16x16x4 -- operands rounded to fp32
// as they enter LDS, fp32 accumulation).
template <typename TS, typename CT, int BM, int BN, int WGM, int WGN, int BK_, int PF = TK_F64_PREFETCH>
__global__ __launch_bounds__(64 * WGM * WGN, (kF64WavesPerEu<BM, BN, BK_>)) void gemm_stream_kernel(GemmArgs args) {
  using TT = F64Tile<BM, BN, WGM, WGN, BK_>;
  using AT = typename MfmaOf<CT>::acc;
  constexpr int NT = TT::NT, BK = TT::BK, TM = TT::TM, TN = TT::TN;
  constexpr int A_TPM = TT::A_TPM, A_LD = TT::A_LD;
  constexpr int ES = sizeof(TS);
  constexpr int GS = MfmaOf<CT>::gs, VS = MfmaOf<CT>::vs;  // column of value v of lane l: GS (l/16) + VS v
  __shared__ CT As[2][BK][BM + TT::APAD];
  __shared__ CT Bs[2][BN][BK + TT::BPAD];

  const TK_CONST GemmTile* tiles = const_ptr(args.tiles);
  const TK_CONST GemmDesc* descs = const_ptr(args.descs);
  const int t_begin = const_ptr(args.wg_first)[blockIdx.x], t_end = const_ptr(args.wg_first)[blockIdx.x + 1];
  if (t_begin >= t_end) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  int wm, wn;
  wave_origin<TT>(wave, &wm, &wn);
  static_assert(BM % 64 == 0 && 64 % BK == 0, "load mapping");
  // wave-uniform parts of the load mapping (A: one k row per instruction;
  // B: 64/BK columns per instruction)
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int a_k = (wv * 64) / BM, a_m0 = (wv * 64) % BM, a_m = a_m0 + lane;
  constexpr int B_NPL = NT / BK;  // columns of B covered per load
  constexpr int B_LDK = BN / B_NPL;
  const int b_c0 = wv * (64 / BK), b_cl = lane / BK, b_k = lane % BK, b_n = b_c0 + b_cl;

  // The workgroup's tiles form one stream of K stages, each tile's stage
  // count rounded up to a multiple of PF (the extra stages load zeros and
  // skip their MFMAs).  A load cursor runs PF + 1 stages ahead of the
  // multiply cursor through a register ring of PF stages and a double
  // buffered LDS stage, across tile boundaries: the first stages of the next
  // tile are in flight before the epilogue of the current one issues its
  // stores, and no tile starts with an empty pipeline.
  auto padded_stages = [&](int t) {
    const GemmTile tt = tiles[t];
    const int n = max(1, (tt.k1 - tt.k0 + BK - 1) / BK);
    return (n + PF - 1) / PF * PF;
  };
  int total = 0;
  for (int t = t_begin; t < t_end; ++t) total += padded_stages(t);

  // Operand loads are raw buffer loads, one resource per load instruction
  // with a wave-uniform base: a load whose offset reaches past the
  // resource's record count reads zero, which pads ragged tile edges, the K
  // tail and the stages past the last tile without branches (so the loads
  // form straight-line code and the waits for them can be counted exactly).
  // A: each instruction of a wave reads 64 consecutive m of one k row; its
  // record count is the number of valid m of that run, or zero past the K
  // range.  B: each instruction reads 64/BK columns of BK consecutive k;
  // invalid lanes get an out-of-range offset.
  // load cursor: tile, stage, stage count and K range of the tile; one
  // resource per operand and stage whose base advances by a whole stage
  // (wave-uniform, scalar registers), and per lane the byte offset of each
  // of its loads inside a stage, fixed for the tile (0x80000000: the lane's
  // row or column lies past M or N, the load reads zero).  A's record count
  // ends at the tile's K range, so its rows past K read zero; B's loads past
  // the K range get the invalid offset.  The offsets stay below
  // BK * lda * 8 and BN * ldb * 8 < 2^31 (the planner checks).
  int l_t = 0, l_s = 0, l_ns = 0, l_k0 = 0, l_kend = 0;
  const char* a_stage = nullptr;
  const char* b_stage = nullptr;
  int64_t a_adv = 0;  // bytes between two stages of A (BK rows)
  int64_t lda8 = 0;
  uint32_t a_voff[A_LD], b_voff[B_LDK];
  auto uni = [](int x) { return __builtin_amdgcn_readfirstlane(x); };
  auto uni64 = [](int64_t x) {
    const uint64_t u = static_cast<uint64_t>(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
  };
  auto load_tile = [&](int t_) {
    const int t = uni(t_);
    l_t = t;
    l_s = 0;
    if (t >= t_end) {  // past the last tile: every later load reads zero
      l_ns = 1 << 30;
      l_kend = l_k0;
      return;
    }
    const GemmTile tile = tiles[t];
    const GemmDesc d = descs[tile.gemm];
    l_ns = uni(padded_stages(t));
    l_k0 = uni(tile.k0);
    l_kend = uni(tile.k1);
    lda8 = uni64(static_cast<int64_t>(d.lda) * ES);
    a_adv = uni64(static_cast<int64_t>(d.lda) * ES * BK);
    const TK_GLOBAL TS* A = buf_ptr<const TS>(args.ptrs, d.a_buf) + d.a + tile.m0 + a_m0 +
                            static_cast<int64_t>(tile.k0 + a_k) * d.lda;
    const TK_GLOBAL TS* B =
        buf_ptr<const TS>(args.ptrs, d.b_buf) + d.b + static_cast<int64_t>(tile.n0 + b_c0) * d.ldb + tile.k0;
    a_stage = reinterpret_cast<const char*>(uni64(reinterpret_cast<int64_t>((const TS*)A)));
    b_stage = reinterpret_cast<const char*>(uni64(reinterpret_cast<int64_t>((const TS*)B)));
    const bool m_ok = lane < d.M - tile.m0 - a_m0;
#pragma unroll
    for (int i = 0; i < A_LD; ++i)
      a_voff[i] = m_ok ? static_cast<uint32_t>((A_TPM * i * d.lda + lane) * ES) : 0x80000000u;
#pragma unroll
    for (int i = 0; i < B_LDK; ++i)
      b_voff[i] = tile.n0 + b_c0 + B_NPL * i + b_cl < d.N
                      ? static_cast<uint32_t>(((B_NPL * i + b_cl) * d.ldb + b_k) * ES)
                      : 0x80000000u;
  };
  TS ra[PF][A_LD], rb[PF][B_LDK];
  // loads the load cursor's stage into ring slot `slot` and advances it
  auto gload_next = [&](int slot) {
    const int k0 = l_k0 + l_s * BK;
    // A rows k0 + a_k + A_TPM i of the K range lie below the record count
    const int64_t rem = static_cast<int64_t>(l_kend - k0 - a_k) * lda8;
    const uint32_t recs = rem <= 0 ? 0u : rem >= 0x7fffffff ? 0x7fffffffu : static_cast<uint32_t>(rem);
    const __amdgpu_buffer_rsrc_t r_a = __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(a_stage), 0, recs, kBufWord3);
#pragma unroll
    for (int i = 0; i < A_LD; ++i) ra[slot][i] = buffer_load<TS>(r_a, a_voff[i]);
    const bool k_ok = k0 + b_k < l_kend;
    const __amdgpu_buffer_rsrc_t r_b =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b_stage), 0, 0x7fffffff, kBufWord3);
#pragma unroll
    for (int i = 0; i < B_LDK; ++i) rb[slot][i] = buffer_load<TS>(r_b, k_ok ? b_voff[i] : 0x80000000u);
    a_stage += a_adv;
    b_stage += BK * ES;
    if (++l_s == l_ns) load_tile(l_t + 1);
  };
  auto lstore = [&](int slot, int buf) {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) As[buf][a_k + A_TPM * i][a_m] = static_cast<CT>(ra[slot][i]);
#pragma unroll
    for (int i = 0; i < B_LDK; ++i) Bs[buf][b_n + B_NPL * i][b_k] = static_cast<CT>(rb[slot][i]);
  };

  AT acc[TM][TN];
  auto compute = [&](int cur) {
#pragma unroll
    for (int j = 0; j < BK / 4; ++j) {
      CT af[TM], bf[TN];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi) af[mi] = As[cur][(BK / 4) * g + j][wm + 16 * mi + l16];
#pragma unroll
      for (int ni = 0; ni < TN; ++ni) bf[ni] = Bs[cur][wn + 16 * ni + l16][(BK / 4) * g + j];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
#pragma unroll
        for (int ni = 0; ni < TN; ++ni)
          acc[mi][ni] = MfmaOf<CT>::mma(bf[ni], af[mi], acc[mi][ni]);
    }
  };

  // multiply cursor: tile ct, its first stage number in the stream, its
  // true stage count, and whether this wave's sub-tile has any valid entry
  // (a wave whose whole sub-tile lies past M or N skips its MFMAs; see
  // wave_origin for why that shortens edge tiles)
  int ct = t_begin, cbase = 0, cnst = 0;
  bool active = false;
  auto compute_tile = [&](int t) {
    const GemmTile tile = tiles[t];
    const GemmDesc d = descs[tile.gemm];
    cnst = max(1, (tile.k1 - tile.k0 + BK - 1) / BK);
    active = tile.m0 + wm < d.M && tile.n0 + wn < d.N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = AT{0, 0, 0, 0};
  };
  compute_tile(ct);

  load_tile(t_begin);
#pragma unroll
  for (int p = 0; p < PF; ++p) gload_next(p);
  lstore(0, 0);
  gload_next(0);
  // stream stage G lives in ring slot G % PF and in LDS buffer G % 2
  for (int G0 = 0; G0 < total; G0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int G = G0 + u;
      __syncthreads();
      lstore((u + 1) % PF, (G + 1) & 1);
      gload_next((u + 1) % PF);
      if (active && G - cbase < cnst) compute(G & 1);
    }
    if (G0 + PF - cbase >= cnst) {
      // tile ct is complete: epilogue, then move the multiply cursor on.
      // The MFMAs take B as their first operand, so each 16x16 accumulator
      // holds the transposed tile: value v of lane l is C[row l % 16][col
      // GS (l/16) + VS v] (the fp64 MFMA places value v of lane l at row
      // l/16 + 4v, column l % 16 of its result, the fp32 one at row
      // 4 (l/16) + v; measured with a lane-layout probe on gfx950).  One
      // store instruction then writes 16 consecutive rows of 4 columns.
      const GemmTile tile = tiles[ct];
      const GemmDesc d = descs[tile.gemm];
      if (tile.nsplit > 1) {
        // partial tile of one K split: stored lane-major for the reduce kernel
        // stored in the accumulator's own type (fp32 accumulators: fp32
        // partials, half the bytes; the reduce widens them exactly)
        CT* mine = reinterpret_cast<CT*>(args.partials) + static_cast<int64_t>(tile.slot0 + tile.split) * (BM * BN);
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int ni = 0; ni < TN; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (tile.m0 + wm + 16 * mi + l16 < d.M && tile.n0 + wn + 16 * ni + GS * g + VS * v < d.N)
                mine[((mi * TN + ni) * 4 + v) * NT + tid] = acc[mi][ni][v];
      } else {
        store_tile_t<TS, AT, TM, TN, VS>(args, d, buf_ptr<TS>(args.ptrs, d.c_buf), tile.m0 + wm + l16,
                                         tile.n0 + wn + GS * g, uni(tile.m0 + wm), uni(tile.n0 + wn), acc);
      }
      // nothing left in flight (see the same wait in gemm_split3_kernel)
      __builtin_amdgcn_s_waitcnt(0x0F70);
      cbase = G0 + PF;
      if (++ct < t_end) compute_tile(ct);
    }
  }
}

// Sum of the K-split partial tiles of the split groups, in split order (a
// fixed order: the result does not depend on which unit finished first),
// then the same epilogue as an unsplit tile.  A flat stream over (group,
// element) pairs: element e of a partial tile is the accumulator value the
// GEMM thread e % NT held as its value number e / NT.
// LAYOUT 0: fp64 arithmetic, transposed accumulators (row lane % 16,
// column lane/16 + 4v); 2: fp32 accumulation (fp32 or split-BF16x3 MFMAs),
// transposed (row lane % 16, column 4 (lane/16) + v).
template <typename TS, int BM, int BN, int WGM, int WGN, int LAYOUT>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs args, const GemmTile* groups, int64_t total) {
  using TT = F64Tile<BM, BN, WGM, WGN>;
  constexpr int NT = TT::NT, TN = TT::TN;
  static_assert((BM * BN) % 256 == 0, "a workgroup's elements must lie in one group");
  for (int64_t x = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; x < total;
       x += static_cast<int64_t>(gridDim.x) * 256) {
    // a workgroup's 256 consecutive elements lie in one group (BM * BN is a
    // multiple of 256), so the group and its tables are uniform: scalar loads
    const int grp = __builtin_amdgcn_readfirstlane(static_cast<int>(x / (BM * BN)));
    const int e = static_cast<int>(x % (BM * BN));
    const int tid = e % NT, val = e / NT;
    const int v = val & 3, t = val >> 2;
    const int mi = t / TN, ni = t % TN;
    const int lane = tid & 63, wave = tid >> 6;
    const GemmTile tile = const_ptr(groups)[grp];
    const GemmDesc d = const_ptr(args.descs)[tile.gemm];
    int wm, wn;
    wave_origin<TT>(wave, &wm, &wn);
    const int r = tile.m0 + wm + 16 * mi + (lane & 15);
    const int c = tile.n0 + wn + 16 * ni + (LAYOUT == 0 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
    if (r >= d.M || c >= d.N) continue;
    // partials in the accumulators' type: fp64 (LAYOUT 0) or fp32 (LAYOUT 2)
    using PT = typename std::conditional<LAYOUT == 0, double, float>::type;
    double sum = 0.0;
    const PT* p = reinterpret_cast<const PT*>(args.partials) + static_cast<int64_t>(tile.slot0) * (BM * BN) + e;
    for (int j = 0; j < tile.nsplit; ++j) sum += static_cast<double>(p[static_cast<int64_t>(j) * (BM * BN)]);
    store_elem<TS>(args, d, buf_ptr<TS>(args.ptrs, d.c_buf), r, c, sum);
  }
}

// ---------------------------------------------------------------------------
// grouped sector GEMM in reduced precision
// ---------------------------------------------------------------------------
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));


// Compensated split-BF16x3 grouped GEMM.  The operand permute has already
// split every value a (rounded to fp32) into hi = bf16(a) and
// lo = bf16(a - hi), stored as two planes with k contiguous: A~ by rows
// (element (m, k) at a + m lda + k), B~ by columns (element (k, n) at
// b + n ldb + k), lda = ldb = K rounded up to 8 with zero padding.  So a
// 16-byte load reads 8 consecutive k of one row of A~ or column of B~, both
// operands stage into LDS as [row][k] with no conversion, and each 16x16x32
// block of the product is lo*hi' + hi*lo' + hi*hi' on the bf16 MFMA with
// fp32 accumulation (the lo*lo' term is dropped).  The pipeline is the one of
// gemm_stream_kernel: every tile of a workgroup is one stream of BK-deep
// stages (each tile's count rounded up to PF), a load cursor PF + 1 stages
// ahead through a register ring, a double-buffered LDS stage, one barrier per
// stage.  Loads are raw buffer loads: rows past M (N) lie past the
// resource's records and k chunks past the tile's K range get an
// out-of-range offset, so both read zero.  The MFMAs take B as the first
// operand, so the accumulators hold the transposed tile (lane l, value v =
// C[l % 16][4 (l/16) + v]) and the epilogue of the fp32 stream kernel
// applies.  LDS rows hold BK = 32 bf16 (64 bytes, four 16-byte chunks)
// with no padding; chunk c of row r sits at position c ^ ((r >> 1) & 3).
// Measured with an LDS probe on gfx950 (SQ_LDS_BANK_CONFLICT): both the
// MFMA operand reads (16 rows, one chunk each) and the staging writes (4
// rows of 4 chunks per 16 lanes) are then conflict free, where rows padded
// by 8 bf16 stalled on conflicts for about half of the LDS-active cycles.
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

// element offset of 16-byte chunk c of row r in the swizzled LDS tile
__device__ __forceinline__ int swz(int r, int c) { return r * 32 + 8 * (c ^ ((r >> 1) & 3)); }

template <typename TS, int BM, int BN, int WGM, int WGN, int BK, int PF = 2>
__global__ __launch_bounds__(64 * WGM * WGN, 2) void gemm_split3_kernel(GemmArgs args) {
  using TT = F64Tile<BM, BN, WGM, WGN, BK>;
  constexpr int NT = TT::NT, TM = TT::TM, TN = TT::TN;
  constexpr int CPR = BK / 8;  // 16-byte chunks of a row per stage
  constexpr int A_CH = BM * CPR, B_CH = BN * CPR;
  constexpr int A_PT = (A_CH + NT - 1) / NT, B_PT = (B_CH + NT - 1) / NT;
  static_assert(BK == 32, "bf16 stage depth (one 16x16x32 MFMA step, swizzled 64-byte rows)");
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM * BK];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][BM * BK];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BN * BK];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][BN * BK];

  const TK_CONST GemmTile* tiles = const_ptr(args.tiles);
  const TK_CONST GemmDesc* descs = const_ptr(args.descs);
  const int t_begin = const_ptr(args.wg_first)[blockIdx.x], t_end = const_ptr(args.wg_first)[blockIdx.x + 1];
  if (t_begin >= t_end) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  int wm, wn;
  wave_origin<TT>(wave, &wm, &wn);
  auto uni = [](int x) { return __builtin_amdgcn_readfirstlane(x); };
  auto uni64 = [](int64_t x) {
    const uint64_t u = static_cast<uint64_t>(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
  };
  auto padded_stages = [&](int t) {
    const GemmTile tt = tiles[t];
    const int n = max(1, (tt.k1 - tt.k0 + BK - 1) / BK);
    return (n + PF - 1) / PF * PF;
  };
  int total = 0;
  for (int t = t_begin; t < t_end; ++t) total += padded_stages(t);

  // load cursor: the tile's resources (hi and lo planes of its A rows and B
  // columns, records = valid rows x ld), its stage count and K range, and
  // this lane's chunk offsets within a stage
  int l_t = 0, l_s = 0, l_ns = 0, l_k0 = 0, l_kend = 0;
  const char *pah = nullptr, *pal = nullptr, *pbh = nullptr, *pbl = nullptr;
  uint32_t abytes = 0, bbytes = 0;
  uint32_t a_off[A_PT], b_off[B_PT];
  int a_kc[A_PT], b_kc[B_PT];
  auto make_rsrc = [](const char* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), 0, bytes, kBufWord3);
  };
  auto uptr = [&](const TK_GLOBAL __bf16* x) {
    return reinterpret_cast<const char*>(uni64(reinterpret_cast<int64_t>((const __bf16*)x)));
  };
  auto load_tile = [&](int t_) {
    const int t = uni(t_);
    l_t = t;
    l_s = 0;
    if (t >= t_end) {  // past the last tile: every later load reads zero
      l_ns = 1 << 30;
      l_kend = l_k0;
      return;
    }
    const GemmTile tile = tiles[t];
    const GemmDesc d = descs[tile.gemm];
    l_ns = uni(padded_stages(t));
    l_k0 = uni(tile.k0);
    l_kend = uni(tile.k1);
    const TK_GLOBAL __bf16* A = (const TK_GLOBAL __bf16*)buf_ptr<const void>(args.ptrs, d.a_buf) + d.a +
                                static_cast<int64_t>(tile.m0) * d.lda;
    const TK_GLOBAL __bf16* B = (const TK_GLOBAL __bf16*)buf_ptr<const void>(args.ptrs, d.b_buf) + d.b +
                                static_cast<int64_t>(tile.n0) * d.ldb;
    abytes = static_cast<uint32_t>(uni(max(0, min(BM, d.M - tile.m0)) * d.lda * 2));
    bbytes = static_cast<uint32_t>(uni(max(0, min(BN, d.N - tile.n0)) * d.ldb * 2));
    pah = uptr(A);
    pal = uptr(A + d.alo);
    pbh = uptr(B);
    pbl = uptr(B + d.blo);
#pragma unroll
    for (int p = 0; p < A_PT; ++p) {
      const int c = tid + p * NT;
      a_kc[p] = 8 * (c % CPR);
      a_off[p] = static_cast<uint32_t>(((c / CPR) * d.lda + a_kc[p]) * 2);
    }
#pragma unroll
    for (int p = 0; p < B_PT; ++p) {
      const int c = tid + p * NT;
      b_kc[p] = 8 * (c % CPR);
      b_off[p] = static_cast<uint32_t>(((c / CPR) * d.ldb + b_kc[p]) * 2);
    }
  };
  u4_t rah_r[PF][A_PT], ral_r[PF][A_PT], rbh_r[PF][B_PT], rbl_r[PF][B_PT];
  auto gload_next = [&](int slot) {
    const int k0 = l_k0 + l_s * BK;
    const __amdgpu_buffer_rsrc_t rah = make_rsrc(pah, abytes), ral = make_rsrc(pal, abytes);
    const __amdgpu_buffer_rsrc_t rbh = make_rsrc(pbh, bbytes), rbl = make_rsrc(pbl, bbytes);
#pragma unroll
    for (int p = 0; p < A_PT; ++p) {
      const bool ok = (A_CH % NT == 0 || tid + p * NT < A_CH) && k0 + a_kc[p] < l_kend;
      const uint32_t off = ok ? a_off[p] + static_cast<uint32_t>(k0 * 2) : 0x80000000u;
      rah_r[slot][p] = __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(rah, off, 0, 0));
      ral_r[slot][p] = __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(ral, off, 0, 0));
    }
#pragma unroll
    for (int p = 0; p < B_PT; ++p) {
      const bool ok = (B_CH % NT == 0 || tid + p * NT < B_CH) && k0 + b_kc[p] < l_kend;
      const uint32_t off = ok ? b_off[p] + static_cast<uint32_t>(k0 * 2) : 0x80000000u;
      rbh_r[slot][p] = __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(rbh, off, 0, 0));
      rbl_r[slot][p] = __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(rbl, off, 0, 0));
    }
    if (++l_s == l_ns) load_tile(l_t + 1);
  };
  auto lstore = [&](int slot, int buf) {
#pragma unroll
    for (int p = 0; p < A_PT; ++p) {
      const int c = tid + p * NT;
      if (A_CH % NT == 0 || c < A_CH) {
        *reinterpret_cast<u4_t*>(&Ah[buf][swz(c / CPR, c % CPR)]) = rah_r[slot][p];
        *reinterpret_cast<u4_t*>(&Al[buf][swz(c / CPR, c % CPR)]) = ral_r[slot][p];
      }
    }
#pragma unroll
    for (int p = 0; p < B_PT; ++p) {
      const int c = tid + p * NT;
      if (B_CH % NT == 0 || c < B_CH) {
        *reinterpret_cast<u4_t*>(&Bh[buf][swz(c / CPR, c % CPR)]) = rbh_r[slot][p];
        *reinterpret_cast<u4_t*>(&Bl[buf][swz(c / CPR, c % CPR)]) = rbl_r[slot][p];
      }
    }
  };

  f4_t acc[TM][TN];
  auto compute = [&](int cur) {
    {
      bf8_t ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi) {
        ah[mi] = *reinterpret_cast<const bf8_t*>(&Ah[cur][swz(wm + 16 * mi + l16, g)]);
        al[mi] = *reinterpret_cast<const bf8_t*>(&Al[cur][swz(wm + 16 * mi + l16, g)]);
      }
#pragma unroll
      for (int ni = 0; ni < TN; ++ni) {
        bh[ni] = *reinterpret_cast<const bf8_t*>(&Bh[cur][swz(wn + 16 * ni + l16, g)]);
        bl[ni] = *reinterpret_cast<const bf8_t*>(&Bl[cur][swz(wn + 16 * ni + l16, g)]);
      }
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
#pragma unroll
        for (int ni = 0; ni < TN; ++ni) {
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[ni], ah[mi], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[ni], al[mi], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[ni], ah[mi], acc[mi][ni], 0, 0, 0);
        }
    }
  };

  int ct = t_begin, cbase = 0, cnst = 0;
  bool active = false;
  auto compute_tile = [&](int t) {
    const GemmTile tile = tiles[t];
    const GemmDesc d = descs[tile.gemm];
    cnst = max(1, (tile.k1 - tile.k0 + BK - 1) / BK);
    active = tile.m0 + wm < d.M && tile.n0 + wn < d.N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  };
  compute_tile(ct);

  load_tile(t_begin);
#pragma unroll
  for (int p = 0; p < PF; ++p) gload_next(p);
  lstore(0, 0);
  gload_next(0);
  for (int G0 = 0; G0 < total; G0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int G = G0 + u;
      __syncthreads();
      lstore((u + 1) % PF, (G + 1) & 1);
      gload_next((u + 1) % PF);
      if (active && G - cbase < cnst) compute(G & 1);
    }
    if (G0 + PF - cbase >= cnst) {
      const GemmTile tile = tiles[ct];
      const GemmDesc d = descs[tile.gemm];
      if (tile.nsplit > 1) {
        // fp32 partials (the accumulators' type; the reduce widens them exactly)
        float* mine = reinterpret_cast<float*>(args.partials) + static_cast<int64_t>(tile.slot0 + tile.split) * (BM * BN);
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int ni = 0; ni < TN; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (tile.m0 + wm + 16 * mi + l16 < d.M && tile.n0 + wn + 16 * ni + 4 * g + v < d.N)
                mine[((mi * TN + ni) * 4 + v) * NT + tid] = acc[mi][ni][v];
      } else {
        store_tile_t<TS, f4_t, TM, TN, 1>(args, d, buf_ptr<TS>(args.ptrs, d.c_buf), tile.m0 + wm + l16,
                                          tile.n0 + wn + 4 * g, __builtin_amdgcn_readfirstlane(tile.m0 + wm),
                                          __builtin_amdgcn_readfirstlane(tile.n0 + wn), acc);
      }
      // The epilogue's table loads are done by now (the stage loads issued
      // before them are too: the counter is in order), but some of their
      // results are never read, and the compiler would otherwise keep those
      // registers pending and make every later stage wait for its own
      // prefetch before the LDS reads.  vmcnt(0): nothing is left in flight.
      __builtin_amdgcn_s_waitcnt(0x0F70);
      cbase = G0 + PF;
      if (++ct < t_end) compute_tile(ct);
    }
  }
}

// ---------------------------------------------------------------------------
// small-K sector GEMMs as an output-stationary stream
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_round(float x) {
  return static_cast<float>(static_cast<__bf16>(x));
}

// MODE 0: arithmetic in the storage type; 1: fp32; 2: two-term bf16 split of
// each operand, three products, fp32 accumulation (the compensated mode).
// sum_k a_k b_k over KK terms in the arithmetic of MODE (see smallk_kernel)
template <int MODE, int KK>
__device__ __forceinline__ double smallk_dot(const double* a, const double* b) {
  if (MODE == 0) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < KK; ++k) s = fma(a[k], b[k], s);
    return s;
  } else if (MODE == 1) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < KK; ++k) s = fmaf(static_cast<float>(a[k]), static_cast<float>(b[k]), s);
    return s;
  } else {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
      const float x = static_cast<float>(a[k]), y = static_cast<float>(b[k]);
      const float xh = bf16_round(x), yh = bf16_round(y);
      const float xl = bf16_round(x - xh), yl = bf16_round(y - yh);
      s = fmaf(xh, yh, s);
      s = fmaf(xh, yl, s);
      s = fmaf(xl, yh, s);
    }
    return s;
  }
}

// Sector GEMMs with K = KK <= 8 fixed at compile time: HBM-bound, no MFMA.
// One workgroup per task (up to kThreads x smallk_rows_per_thread(KK) rows of
// one row channel); thread t owns rows t, t + kThreads, ...: the KK values of
// A~ of all its rows are loaded before any is used (consecutive rows are
// consecutive in A~, so the loads are coalesced; several rows per thread
// keep more loads in flight when KK is small), then the task's columns are
// walked in order; B~ values, channel tables and pair descriptors are the
// same for every lane (scalar loads), and each output is written from
// registers (consecutive rows of a channel land at a stride of the output's
// row-leg layout, unit stride when its first leg leads the output block).
// MODE 0: fp64 arithmetic (fp64 tensors); 1: fp32 (fp32 tensors, or the fp32
// mode); 2: two-term bf16 split of each operand, three products, fp32
// accumulation (the compensated mode).
template <typename T, int MODE, int KK>
__global__ __launch_bounds__(kThreads) void smallk_kernel(const SmallKTask* __restrict__ tasks,
                                                          const SkChan* __restrict__ chans,
                                                          const PairDesc* __restrict__ pairs, Ptrs P, double alpha,
                                                          double beta) {
  constexpr int RT = smallk_rows_per_thread(KK);
  const SmallKTask tk = const_ptr(tasks)[blockIdx.x];
  const TK_CONST SkChan* ch = const_ptr(chans);
  const TK_CONST PairDesc* pr = const_ptr(pairs);
  const TK_GLOBAL T* __restrict__ A = buf_ptr<const T>(P, tk.a_buf) + tk.a;
  const TK_CONST T* Bc = const_ptr((const T*)(buf_ptr<const T>(P, tk.b_buf) + tk.b));
  TK_GLOBAL T* __restrict__ D = buf_ptr<T>(P, tk.dst_buf);
  bool ok[RT];
  double a[RT][KK];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int row = threadIdx.x + q * kThreads;
    ok[q] = row < tk.rows;
    const int rr = ok[q] ? row : tk.rows - 1;
#pragma unroll
    for (int k = 0; k < KK; ++k) a[q][k] = static_cast<double>(A[rr + static_cast<int64_t>(k) * tk.lda]);
  }
  // leg indices of each row inside its channel (colex, first leg fastest)
  int ri[RT][4];
  {
    const SkChan rc = ch[tk.rchan];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const int row = threadIdx.x + q * kThreads;
      int rem = tk.r0 + (ok[q] ? row : tk.rows - 1);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        ri[q][l] = 0;
        if (l < tk.nrleg) {
          ri[q][l] = rem % rc.dim[l];
          rem /= rc.dim[l];
        }
      }
    }
  }
  int j = tk.cchan, pi = tk.pair;
  SkChan cc = ch[j];
  PairDesc pd = pr[pi];
  int64_t rowpart[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    rowpart[q] = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) rowpart[q] += static_cast<int64_t>(ri[q][l]) * pd.S[l];
  }
  // column leg indices of the current column (colex counter, first leg
  // fastest), started at column c0 of channel cchan
  int ci[4] = {0, 0, 0, 0};
  {
    int rem = tk.c0;
#pragma unroll
    for (int l = 0; l < 4; ++l)
      if (l < tk.ncleg) {
        ci[l] = rem % cc.dim[l];
        rem /= cc.dim[l];
      }
  }
  int c = tk.c0;
  for (int n = 0; n < tk.ncols; ++n) {
    if (c == cc.count) {  // next column channel (uniform)
      ++j;
      ++pi;
      c = 0;
      cc = ch[j];
      pd = pr[pi];
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        rowpart[q] = 0;
#pragma unroll
        for (int l = 0; l < 4; ++l) rowpart[q] += static_cast<int64_t>(ri[q][l]) * pd.S[l];
      }
#pragma unroll
      for (int l = 0; l < 4; ++l) ci[l] = 0;
    }
    int64_t colpart = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) colpart += static_cast<int64_t>(ci[l]) * pd.S[4 + l];
    double b[KK];
    const int64_t bo = static_cast<int64_t>(tk.bcol + n) * tk.ldb;
#pragma unroll
    for (int k = 0; k < KK; ++k) b[k] = static_cast<double>(Bc[bo + k]);
    const double scale = alpha * static_cast<double>(pd.sign);
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      double v = scale * smallk_dot<MODE, KK>(a[q], b);
      const int64_t x = pd.base + rowpart[q] + colpart;
      if (ok[q]) {
        if (beta != 0.0) v += beta * static_cast<double>(D[x]);
        D[x] = static_cast<T>(v);
      }
    }
    ++c;
#pragma unroll
    for (int l = 0; l < 4; ++l) {  // advance the colex counter
      if (l < tk.ncleg && ++ci[l] < cc.dim[l]) break;
      if (l < tk.ncleg) ci[l] = 0;
    }
  }
}

// Small-K sectors with many columns: output-stationary.  Tasks are chunks
// of one output block, enumerated in the output's own order (so the stores
// of consecutive lanes are consecutive when the block is contiguous); each
// element's row inside the row channel and column inside the column channel
// come from its output leg indices, and its KK values of A~ and B~ (small,
// read from cache) are combined as in smallk_kernel.  A workgroup with one
// task spreads it over all its threads, one with several gives each wave its
// own tasks.
// a[i & 3] as a select chain: a dynamic index would put the array in
// scratch memory
template <typename V>
__device__ __forceinline__ V pick4(const V* a, int i) {
  i &= 3;
  return i == 0 ? a[0] : i == 1 ? a[1] : i == 2 ? a[2] : a[3];
}

template <typename T, int MODE, int KK>
__device__ __forceinline__ void smallk_block(const SkBlockTask& tk, const SkChan& rc, const SkChan& cc,
                                             const PairDesc& pd, int start, int count, const Ptrs& P, double alpha,
                                             double beta, int lt, int nthr) {
  int32_t dim[8], ra[8], cb[8], so[8];
  uint32_t mag[8];
  int shr[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    dim[o] = 1;
    mag[o] = 0;
    shr[o] = 0;
    ra[o] = cb[o] = so[o] = 0;
    if (o < tk.nout) {
      const int l = (tk.order >> (4 * o)) & 15;
      int32_t stride = 1;
      if (l < tk.nrleg) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < l) stride *= rc.dim[q];
        dim[o] = pick4(rc.dim, l);
        mag[o] = pick4(rc.mag, l);
        shr[o] = pick4(rc.shr, l);
        ra[o] = stride;
        so[o] = pick4(pd.S, l);
      } else {
        const int m = l - tk.nrleg;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < m) stride *= cc.dim[q];
        dim[o] = pick4(cc.dim, m);
        mag[o] = pick4(cc.mag, m);
        shr[o] = pick4(cc.shr, m);
        cb[o] = stride;
        so[o] = pick4(pd.S + 4, m);
      }
    }
  }
  const TK_GLOBAL T* __restrict__ A = buf_ptr<const T>(P, tk.a_buf) + tk.a;
  const TK_GLOBAL T* __restrict__ B = buf_ptr<const T>(P, tk.b_buf) + tk.b;
  TK_GLOBAL T* __restrict__ D = buf_ptr<T>(P, tk.dst_buf) + pd.base;
  const double scale = alpha * static_cast<double>(pd.sign);
  constexpr int U = 4;
  for (int e0 = 0; e0 < count; e0 += nthr * U) {
    int64_t r[U], c[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t lin = static_cast<uint32_t>(start + min(e0 + u * nthr + lt, count - 1));
      int64_t rr = 0, cc2 = 0, xx = 0;
#pragma unroll
      for (int o = 0; o < 8; ++o)
        if (o < tk.nout) {
          const uint32_t q = static_cast<uint32_t>((static_cast<uint64_t>(lin) * mag[o]) >> shr[o]);
          const uint32_t i = lin - q * static_cast<uint32_t>(dim[o]);
          lin = q;
          rr += static_cast<int64_t>(i) * ra[o];
          cc2 += static_cast<int64_t>(i) * cb[o];
          xx += static_cast<int64_t>(i) * so[o];
        }
      r[u] = rr;
      c[u] = (cc2 + cc.off) * tk.ldb;
      x[u] = xx;
    }
    double av[U][KK], bv[U][KK];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < KK; ++k) {
        av[u][k] = static_cast<double>(A[r[u] + static_cast<int64_t>(k) * tk.lda]);
        bv[u][k] = static_cast<double>(B[c[u] + k]);
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e0 + u * nthr + lt >= count) continue;
      double v = scale * smallk_dot<MODE, KK>(av[u], bv[u]);
      if (beta != 0.0) v += beta * static_cast<double>(D[x[u]]);
      D[x[u]] = static_cast<T>(v);
    }
  }
}

// One task: a chunk of one block (nblk <= 1), or blocks b0, b0 + bstep, ...
// of a strip, each whole; the next block's channel record and pair are
// read before the current block is written, so their latency overlaps it.
template <typename T, int MODE, int KK>
__device__ __forceinline__ void smallk_strip(const SkBlockTask& tk, const TK_CONST SkChan* ch,
                                             const TK_CONST PairDesc* pr, const Ptrs& P, double alpha, double beta,
                                             int lt, int nthr, int b0, int bstep) {
  const SkChan rc = ch[tk.rchan];
  if (tk.nblk <= 1) {
    const SkChan cc = ch[tk.cchan];
    const PairDesc pd = pr[tk.pair];
    smallk_block<T, MODE, KK>(tk, rc, cc, pd, tk.start, tk.count, P, alpha, beta, lt, nthr);
    return;
  }
  if (b0 >= tk.nblk) return;
  SkChan cn = ch[tk.cchan + b0];
  PairDesc pn = pr[tk.pair + b0];
  for (int b = b0; b < tk.nblk; b += bstep) {
    const SkChan cc = cn;
    const PairDesc pd = pn;
    if (b + bstep < tk.nblk) {
      cn = ch[tk.cchan + b + bstep];
      pn = pr[tk.pair + b + bstep];
    }
    smallk_block<T, MODE, KK>(tk, rc, cc, pd, 0, rc.count * cc.count, P, alpha, beta, lt, nthr);
  }
}

// A workgroup holding one task: a strip is split over the waves by block,
// a single block over all threads; one holding several tasks gives each
// wave its own tasks.
template <typename T, int MODE, int KK>
__global__ __launch_bounds__(kThreads) void smallk_blocks_kernel(const SkBlockTask* __restrict__ tasks,
                                                                 const int32_t* __restrict__ wg_first,
                                                                 const SkChan* __restrict__ chans,
                                                                 const PairDesc* __restrict__ pairs, Ptrs P,
                                                                 double alpha, double beta) {
  const TK_CONST SkChan* ch = const_ptr(chans);
  const TK_CONST PairDesc* pr = const_ptr(pairs);
  const int t0 = const_ptr(wg_first)[blockIdx.x], t1 = const_ptr(wg_first)[blockIdx.x + 1];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t1 - t0 == 1) {
    const SkBlockTask tk = const_ptr(tasks)[t0];
    if (tk.nblk > 1)
      smallk_strip<T, MODE, KK>(tk, ch, pr, P, alpha, beta, lane, 64, wave, kThreads / 64);
    else
      smallk_strip<T, MODE, KK>(tk, ch, pr, P, alpha, beta, threadIdx.x, kThreads, 0, 1);
    return;
  }
  for (int t = t0 + wave; t < t1; t += kThreads / 64) {
    const SkBlockTask tk = const_ptr(tasks)[t];
    smallk_strip<T, MODE, KK>(tk, ch, pr, P, alpha, beta, lane, 64, 0, 1);
  }
}

// Output runs: workgroup w covers elements wstart[w] .. wstart[w+1]-1 of the
// concatenated runs of one K.  Its runs (at most kRunMax + 1) are staged in
// LDS with their block's operand pointers, sign, A~ stride and dimensions,
// and an index map gives each element its run.  The element splits its
// linear index over the dimensions (32-bit multiply-high division, 24-bit
// products) and takes the K-term dot product of its row of A~ and column of
// B~.  Consecutive threads write consecutive elements of C however small the
// blocks are.
template <typename T, int MODE, int KK>
__global__ __launch_bounds__(kThreads) void smallk_runs_kernel(const SkRun* __restrict__ runs, int nruns,
                                                               const int32_t* __restrict__ first,
                                                               const int64_t* __restrict__ wstart,
                                                               const SkRunShape* __restrict__ shapes, Ptrs P,
                                                               double alpha, double beta) {
  static_assert(kRunMax < 255, "run index map is 8-bit");
  __shared__ TK_GLOBAL T* s_p[kRunMax + 1];
  __shared__ const TK_GLOBAL T* s_a[kRunMax + 1];
  __shared__ const TK_GLOBAL T* s_b[kRunMax + 1];
  __shared__ int4 s_i[kRunMax + 1];  // dimensions, lin0 - relative start, lda, sign bits
  __shared__ SkRunDim s_dim[kRunMax + 1][8];
  __shared__ int32_t s_r[kRunMax + 1];
  __shared__ __align__(16) uint8_t s_idx[kRunChunk];
  __shared__ uint32_t s_wmax[kThreads / 64];
  const int64_t c0 = const_ptr(wstart)[blockIdx.x], c1 = const_ptr(wstart)[blockIdx.x + 1];
  const int n = static_cast<int>(c1 - c0);
  const int r0 = const_ptr(first)[blockIdx.x];
  const int r1 = min(nruns, const_ptr(first)[blockIdx.x + 1] + 1);
  const int nr = min(r1 - r0, kRunMax + 1);
  for (int i = threadIdx.x; i < nr; i += kThreads) {
    const SkRun rn = runs[r0 + i];
    const int64_t rel = rn.vstart - c0;  // <= 0 for run 0, in (0, n] for the others
    s_r[i] = static_cast<int32_t>(max<int64_t>(rel, 0));
    s_p[i] = buf_ptr_lane<T>(P, rn.buf) + (rn.off - rel);
    s_a[i] = buf_ptr_lane<const T>(P, rn.a_buf) + rn.a;
    s_b[i] = buf_ptr_lane<const T>(P, rn.b_buf) + rn.b;
    s_i[i] = make_int4(shapes[rn.shape].nd, static_cast<int32_t>(rn.lin0 - rel), rn.lda, __float_as_int(rn.sign));
  }
  // the dimensions: 8 records of 16 bytes per run, one per thread in turn
  for (int t = threadIdx.x; t < nr * 8; t += kThreads) {
    const int i = t >> 3;
    s_dim[i][t & 7] = shapes[runs[r0 + i].shape].dim[t & 7];
  }
  __syncthreads();
  if (nr > 1) chunk_range_map<kRunChunk, uint8_t>(s_idx, s_wmax, s_r, nr, n);
  constexpr int U = KK <= 2 ? 4 : 2;
  for (int e0 = 0; e0 < n; e0 += kThreads * U) {
    int id[U];
    uint32_t ao[U], bo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = min(e0 + u * kThreads + static_cast<int>(threadIdx.x), n - 1);
      const int l = nr > 1 ? s_idx[e] : 0;
      id[u] = l;
      const int4 inf = s_i[l];
      uint32_t lin = static_cast<uint32_t>(inf.y + e);
      uint32_t a = 0, b = 0;
#pragma unroll
      for (int o = 0; o < 8; ++o)
        if (o < inf.x) {
          const SkRunDim d = s_dim[l][o];
          const uint32_t q = __umulhi(lin, d.mag) >> (d.dimshr >> 24);
          const uint32_t i = lin - __umul24(q, d.dimshr & 0xffffffu);
          lin = q;
          a += __umul24(i, d.sa);
          b += __umul24(i, d.sb);
        }
      ao[u] = a;
      bo[u] = b;
    }
    double av[U][KK], bv[U][KK];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const TK_GLOBAL T* A = s_a[id[u]] + ao[u];
      const TK_GLOBAL T* B = s_b[id[u]] + bo[u];
      const int lda = s_i[id[u]].z;
#pragma unroll
      for (int k = 0; k < KK; ++k) {
        av[u][k] = static_cast<double>(A[static_cast<int64_t>(k) * lda]);
        bv[u][k] = static_cast<double>(B[k]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kThreads + static_cast<int>(threadIdx.x);
      if (e >= n) continue;
      const float sg = __int_as_float(s_i[id[u]].w);
      double x = alpha * static_cast<double>(sg) * smallk_dot<MODE, KK>(av[u], bv[u]);
      TK_GLOBAL T* d = s_p[id[u]] + e;
      if (beta != 0.0) x += beta * static_cast<double>(*d);
      *d = static_cast<T>(x);
    }
  }
}

// ---------------------------------------------------------------------------
// scratch memory of the allocation-free contraction entry point: one array
// per device, held from the code object's load until the process ends.  In
// host code its name stands for a host-side shadow, never a device address:
// host code uses only the address scratch_address returns.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** out) { return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)); }

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_zero_ranges(int dtype, const ZeroRange* ranges, int nranges, const int32_t* first,
                              const int64_t* wstart, int nwg, const Ptrs& ptrs, double beta, hipStream_t stream) {
  if (nwg <= 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(zero_ranges_kernel<double>, dim3(nwg), dim3(kThreads), 0, stream, ranges, nranges, first,
                       wstart, ptrs, beta);
  else
    hipLaunchKernelGGL(zero_ranges_kernel<float>, dim3(nwg), dim3(kThreads), 0, stream, ranges, nranges, first,
                       wstart, ptrs, beta);
  return hipGetLastError();
}

hipError_t launch_trace(int dtype, const TraceTask* tasks, const int32_t* wg_first, int nwg,
                        const TraceContrib* contribs, const Ptrs& ptrs, double alpha, double beta, bool gather,
                        hipStream_t stream) {
  if (nwg <= 0) return hipSuccess;
  const auto kernel = dtype == 0 ? (gather ? trace_kernel<double, true> : trace_kernel<double, false>)
                                 : (gather ? trace_kernel<float, true> : trace_kernel<float, false>);
  hipLaunchKernelGGL(kernel, dim3(nwg), dim3(kThreads), 0, stream, tasks, wg_first, contribs, ptrs, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_svd_init(const SvdSector* secs, int nsec, const double* X, double* ws, hipStream_t stream) {
  if (nsec <= 0) return hipSuccess;
  hipLaunchKernelGGL(svd_init_kernel, dim3(nsec), dim3(kSvdThreads), 0, stream, secs, X, ws);
  return hipGetLastError();
}

hipError_t launch_svd_round(const SvdItem* items, int nitems, const SvdSector* secs, double* ws, const int32_t* prev,
                            int32_t* flag, int sweep, double tol, hipStream_t stream) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(svd_round_kernel, dim3(nitems), dim3(kSvdRoundThreads), 0, stream, items, secs, ws, prev, flag,
                     sweep, tol);
  return hipGetLastError();
}

hipError_t launch_svd_finish(const SvdSector* secs, int nsec, double* ws, hipStream_t stream) {
  if (nsec <= 0) return hipSuccess;
  hipLaunchKernelGGL(svd_finish_kernel, dim3(nsec), dim3(kSvdThreads), 0, stream, secs, ws);
  return hipGetLastError();
}

hipError_t launch_permute_tiles(int dtype, const TileTask* tiles, int ntiles, const Ptrs& ptrs, double alpha,
                                double beta, hipStream_t stream, bool split) {
  if (ntiles <= 0) return hipSuccess;
  if (dtype == 0 && split)
    hipLaunchKernelGGL((permute_tile_kernel<double, true>), dim3(ntiles), dim3(kThreads), 0, stream, tiles, ptrs,
                       alpha, beta);
  else if (dtype == 0)
    hipLaunchKernelGGL((permute_tile_kernel<double, false>), dim3(ntiles), dim3(kThreads), 0, stream, tiles, ptrs,
                       alpha, beta);
  else if (split)
    hipLaunchKernelGGL((permute_tile_kernel<float, true>), dim3(ntiles), dim3(kThreads), 0, stream, tiles, ptrs,
                       alpha, beta);
  else
    hipLaunchKernelGGL((permute_tile_kernel<float, false>), dim3(ntiles), dim3(kThreads), 0, stream, tiles, ptrs,
                       alpha, beta);
  return hipGetLastError();
}

hipError_t launch_permute(int dtype, const PermTask* tasks, const int32_t* wg_first, int nwg,
                          const Ptrs& ptrs, double alpha, double beta, hipStream_t stream, bool split) {
  if (nwg <= 0) return hipSuccess;
  if (dtype == 0 && split)
    hipLaunchKernelGGL((permute_kernel<double, true>), dim3(nwg), dim3(kThreads), 0, stream, tasks, wg_first,
                       ptrs, alpha, beta);
  else if (dtype == 0)
    hipLaunchKernelGGL((permute_kernel<double, false>), dim3(nwg), dim3(kThreads), 0, stream, tasks, wg_first,
                       ptrs, alpha, beta);
  else if (split)
    hipLaunchKernelGGL((permute_kernel<float, true>), dim3(nwg), dim3(kThreads), 0, stream, tasks, wg_first,
                       ptrs, alpha, beta);
  else
    hipLaunchKernelGGL((permute_kernel<float, false>), dim3(nwg), dim3(kThreads), 0, stream, tasks, wg_first,
                       ptrs, alpha, beta);
  return hipGetLastError();
}

template <typename T, int MODE>
static void launch_smallk_k(int K, const SmallKTask* tasks, int ntasks, const SkChan* chans, const PairDesc* pairs,
                            const Ptrs& ptrs, double alpha, double beta, hipStream_t stream) {
  switch (K) {
#define TK_SK_CASE(KK_)                                                                                     \
  case KK_:                                                                                                 \
    hipLaunchKernelGGL((smallk_kernel<T, MODE, KK_>), dim3(ntasks), dim3(kThreads), 0, stream, tasks, chans, \
                       pairs, ptrs, alpha, beta);                                                           \
    break;
    TK_SK_CASE(1) TK_SK_CASE(2) TK_SK_CASE(3) TK_SK_CASE(4) TK_SK_CASE(5) TK_SK_CASE(6) TK_SK_CASE(7) TK_SK_CASE(8)
#undef TK_SK_CASE
    default:
      break;
  }
}

template <typename T, int MODE>
static void launch_smallk_blocks_k(int K, const SkBlockTask* tasks, const int32_t* wg_first, int nwg,
                                   const SkChan* chans, const PairDesc* pairs, const Ptrs& ptrs, double alpha,
                                   double beta, hipStream_t stream) {
  switch (K) {
#define TK_SKB_CASE(KK_)                                                                                        \
  case KK_:                                                                                                     \
    hipLaunchKernelGGL((smallk_blocks_kernel<T, MODE, KK_>), dim3(nwg), dim3(kThreads), 0, stream, tasks,       \
                       wg_first, chans, pairs, ptrs, alpha, beta);                                              \
    break;
    TK_SKB_CASE(1) TK_SKB_CASE(2) TK_SKB_CASE(3) TK_SKB_CASE(4) TK_SKB_CASE(5) TK_SKB_CASE(6) TK_SKB_CASE(7)
    TK_SKB_CASE(8)
#undef TK_SKB_CASE
    default:
      break;
  }
}

hipError_t launch_smallk_blocks(int dtype, int precision, int K, const SkBlockTask* tasks, const int32_t* wg_first,
                                int nwg, const SkChan* chans, const PairDesc* pairs, const Ptrs& ptrs, double alpha,
                                double beta, hipStream_t stream) {
  if (nwg <= 0) return hipSuccess;
  if (K < 1 || K > 8) return hipErrorInvalidValue;
  if (dtype == 0) {
    if (precision == 0)
      launch_smallk_blocks_k<double, 0>(K, tasks, wg_first, nwg, chans, pairs, ptrs, alpha, beta, stream);
    else if (precision == 1)
      launch_smallk_blocks_k<double, 1>(K, tasks, wg_first, nwg, chans, pairs, ptrs, alpha, beta, stream);
    else
      launch_smallk_blocks_k<double, 2>(K, tasks, wg_first, nwg, chans, pairs, ptrs, alpha, beta, stream);
  } else {
    if (precision == 2)
      launch_smallk_blocks_k<float, 2>(K, tasks, wg_first, nwg, chans, pairs, ptrs, alpha, beta, stream);
    else
      launch_smallk_blocks_k<float, 1>(K, tasks, wg_first, nwg, chans, pairs, ptrs, alpha, beta, stream);
  }
  return hipGetLastError();
}

template <typename T, int MODE>
static void launch_smallk_runs_k(int K, const SkRun* runs, int nruns, const int32_t* first, const int64_t* wstart,
                                 int nwg, const SkRunShape* shapes, const Ptrs& ptrs, double alpha, double beta,
                                 hipStream_t stream) {
  switch (K) {
#define TK_SKR_CASE(KK_)                                                                                        \
  case KK_:                                                                                                     \
    hipLaunchKernelGGL((smallk_runs_kernel<T, MODE, KK_>), dim3(nwg), dim3(kThreads), 0, stream, runs, nruns,   \
                       first, wstart, shapes, ptrs, alpha, beta);                                               \
    break;
    TK_SKR_CASE(1) TK_SKR_CASE(2) TK_SKR_CASE(3) TK_SKR_CASE(4) TK_SKR_CASE(5) TK_SKR_CASE(6) TK_SKR_CASE(7)
    TK_SKR_CASE(8)
#undef TK_SKR_CASE
    default:
      break;
  }
}

hipError_t launch_smallk_runs(int dtype, int precision, int K, const SkRun* runs, int nruns, const int32_t* first,
                              const int64_t* wstart, int nwg, const SkRunShape* shapes, const Ptrs& ptrs, double alpha,
                              double beta, hipStream_t stream) {
  if (nwg <= 0) return hipSuccess;
  if (K < 1 || K > 8) return hipErrorInvalidValue;
  if (dtype == 0) {
    if (precision == 0)
      launch_smallk_runs_k<double, 0>(K, runs, nruns, first, wstart, nwg, shapes, ptrs, alpha, beta, stream);
    else if (precision == 1)
      launch_smallk_runs_k<double, 1>(K, runs, nruns, first, wstart, nwg, shapes, ptrs, alpha, beta, stream);
    else
      launch_smallk_runs_k<double, 2>(K, runs, nruns, first, wstart, nwg, shapes, ptrs, alpha, beta, stream);
  } else {
    if (precision == 2)
      launch_smallk_runs_k<float, 2>(K, runs, nruns, first, wstart, nwg, shapes, ptrs, alpha, beta, stream);
    else
      launch_smallk_runs_k<float, 1>(K, runs, nruns, first, wstart, nwg, shapes, ptrs, alpha, beta, stream);
  }
  return hipGetLastError();
}

hipError_t launch_smallk(int dtype, int precision, int K, const SmallKTask* tasks, int ntasks, const SkChan* chans,
                         const PairDesc* pairs, const Ptrs& ptrs, double alpha, double beta, hipStream_t stream) {
  if (ntasks <= 0) return hipSuccess;
  if (K < 1 || K > 8) return hipErrorInvalidValue;
  if (dtype == 0) {
    if (precision == 0) launch_smallk_k<double, 0>(K, tasks, ntasks, chans, pairs, ptrs, alpha, beta, stream);
    else if (precision == 1) launch_smallk_k<double, 1>(K, tasks, ntasks, chans, pairs, ptrs, alpha, beta, stream);
    else launch_smallk_k<double, 2>(K, tasks, ntasks, chans, pairs, ptrs, alpha, beta, stream);
  } else {
    if (precision == 2) launch_smallk_k<float, 2>(K, tasks, ntasks, chans, pairs, ptrs, alpha, beta, stream);
    else launch_smallk_k<float, 1>(K, tasks, ntasks, chans, pairs, ptrs, alpha, beta, stream);
  }
  return hipGetLastError();
}

// Tile configurations of the grouped GEMM: (tile_m, tile_n, stage depth) and
// the wave grid that covers the tile.  The bf16 kernel needs a depth of 32.
#define TK_GEMM_SHAPES(X)                                                                             \
  X(128, 128, 16, 2, 4) X(128, 128, 32, 2, 4) X(128, 64, 16, 2, 2) X(128, 64, 32, 2, 2)              \
  X(64, 128, 16, 2, 4) X(64, 128, 32, 2, 4) X(64, 64, 16, 2, 2) X(64, 64, 32, 2, 2)

struct TileShape {
  int m, n, k;
};
static const TileShape kTiles[] = {
#define TK_SHAPE_ENTRY(BM_, BN_, BK_, WM_, WN_) {BM_, BN_, BK_},
    TK_GEMM_SHAPES(TK_SHAPE_ENTRY)
#undef TK_SHAPE_ENTRY
};

int num_tile_shapes() { return static_cast<int>(sizeof(kTiles) / sizeof(kTiles[0])); }
void tile_shape(int i, int* tm, int* tn, int* tk) {
  *tm = kTiles[i].m;
  *tn = kTiles[i].n;
  *tk = kTiles[i].k;
}

// compute kind: 0 fp64 MFMA, 1 fp32 MFMA, 2 split-bf16x3
static int compute_kind(int dtype, int precision) {
  if (precision == 2) return 2;
  if (dtype == 1 || precision == 1) return 1;
  return 0;
}

bool gemm_tile_supported(int dtype, int precision, int tile_m, int tile_n, int tile_k) {
  if (dtype < 0 || dtype > 1 || precision < 0 || precision > 2) return false;
  if (compute_kind(dtype, precision) == 2 && tile_k % 32 != 0) return false;
  for (const auto& t : kTiles)
    if (t.m == tile_m && t.n == tile_n && t.k == tile_k) return true;
  return false;
}

template <typename TS, int BM, int BN, int WM, int WN, int BK>
static void launch_gemm_kind(int kind, const GemmArgs& args, int nwg, hipStream_t stream) {
  const dim3 grid(nwg), block(64 * WM * WN);
  if (kind == 0) {
    if constexpr (sizeof(TS) == 8)
      hipLaunchKernelGGL((gemm_stream_kernel<double, double, BM, BN, WM, WN, BK>), grid, block, 0, stream, args);
  } else if (kind == 1) {
    hipLaunchKernelGGL((gemm_stream_kernel<TS, float, BM, BN, WM, WN, BK>), grid, block, 0, stream, args);
  } else {
    if constexpr (BK % 32 == 0)
      hipLaunchKernelGGL((gemm_split3_kernel<TS, BM, BN, WM, WN, BK>), grid, block, 0, stream, args);
  }
}

hipError_t launch_gemm(int dtype, int precision, int tile_m, int tile_n, int tile_k, const GemmArgs& args, int nwg,
                       hipStream_t stream) {
  if (nwg <= 0) return hipSuccess;
  if (!gemm_tile_supported(dtype, precision, tile_m, tile_n, tile_k)) return hipErrorInvalidValue;
  const int kind = compute_kind(dtype, precision);
#define TK_GEMM_CASE(BM_, BN_, BK_, WM_, WN_)                                           \
  if (tile_m == BM_ && tile_n == BN_ && tile_k == BK_) {                                \
    if (dtype == 0)                                                                     \
      launch_gemm_kind<double, BM_, BN_, WM_, WN_, BK_>(kind, args, nwg, stream);       \
    else                                                                                \
      launch_gemm_kind<float, BM_, BN_, WM_, WN_, BK_>(kind, args, nwg, stream);        \
    return hipGetLastError();                                                           \
  }
  TK_GEMM_SHAPES(TK_GEMM_CASE)
#undef TK_GEMM_CASE
  return hipErrorInvalidValue;
}

template <typename TS, int BM, int BN, int WM, int WN, int BK>
static int blocks_per_cu_kind(int kind) {
  int n = 0;
  hipError_t e = hipSuccess;
  if (kind == 0) {
    if constexpr (sizeof(TS) == 8)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_stream_kernel<double, double, BM, BN, WM, WN, BK>,
                                                       64 * WM * WN, 0);
  } else if (kind == 1) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_stream_kernel<TS, float, BM, BN, WM, WN, BK>,
                                                     64 * WM * WN, 0);
  } else {
    if constexpr (BK % 32 == 0)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_split3_kernel<TS, BM, BN, WM, WN, BK>, 64 * WM * WN,
                                                       0);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n < 1 ? 1 : n;
}

int gemm_blocks_per_cu(int dtype, int precision, int tile_m, int tile_n, int tile_k) {
  if (!gemm_tile_supported(dtype, precision, tile_m, tile_n, tile_k)) return 1;
  const int kind = compute_kind(dtype, precision);
#define TK_OCC_CASE(BM_, BN_, BK_, WM_, WN_)                                                       \
  if (tile_m == BM_ && tile_n == BN_ && tile_k == BK_)                                             \
    return dtype == 0 ? blocks_per_cu_kind<double, BM_, BN_, WM_, WN_, BK_>(kind)                  \
                      : blocks_per_cu_kind<float, BM_, BN_, WM_, WN_, BK_>(kind);
  TK_GEMM_SHAPES(TK_OCC_CASE)
#undef TK_OCC_CASE
  return 1;
}

hipError_t launch_splitk_reduce(int dtype, int precision, int tile_m, int tile_n, int tile_k, const GemmArgs& args,
                                const GemmTile* groups, int ngroups, hipStream_t stream) {
  if (ngroups <= 0) return hipSuccess;
  if (!gemm_tile_supported(dtype, precision, tile_m, tile_n, tile_k)) return hipErrorInvalidValue;
  const int64_t total = static_cast<int64_t>(ngroups) * tile_m * tile_n;
  const unsigned nblk = static_cast<unsigned>(std::min<int64_t>((total + 255) / 256, 65536));
  const int kind = compute_kind(dtype, precision);
#define TK_RED_LAUNCH(TS_, L_, BM_, BN_, WM_, WN_)                                                               \
  hipLaunchKernelGGL((splitk_reduce_kernel<TS_, BM_, BN_, WM_, WN_, L_>), dim3(nblk), dim3(256), 0, stream, args, \
                     groups, total)
#define TK_RED_CASE(BM_, BN_, BK_, WM_, WN_)                                                   \
  if (tile_m == BM_ && tile_n == BN_ && tile_k == BK_) {                                       \
    if (dtype == 0 && kind == 0) {                                                             \
      TK_RED_LAUNCH(double, 0, BM_, BN_, WM_, WN_);                                                                \
    } else if (dtype == 0) {                                                                   \
      TK_RED_LAUNCH(double, 2, BM_, BN_, WM_, WN_);                                                                \
    } else {                                                                                   \
      TK_RED_LAUNCH(float, 2, BM_, BN_, WM_, WN_);                                                                 \
    }                                                                                          \
    return hipGetLastError();                                                                  \
  }
  TK_GEMM_SHAPES(TK_RED_CASE)
#undef TK_RED_CASE
#undef TK_RED_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace tk
