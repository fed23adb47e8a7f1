// Internal descriptors shared by the host planner (tk_host.cpp) and the
// device kernels (tk_kernels.hip).  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace tk {

constexpr int kMaxDims = 8;   // dims of one block task after merging
constexpr int kPermChunk = 4096;  // elements of one block task (a workgroup visit)
constexpr int kThreads = 256;

// Buffer ids used by task descriptors.  A plan reads/writes at most these
// eight buffers (operands, result, workspaces for A~, B~ and, when the
// output permute cannot be fused, C~, and the split-BF16x3 operand planes of
// A~ and B~); a batch offsets them by kBufsPerPlan per member plan.
enum BufId : int16_t {
  kBufA = 0, kBufB = 1, kBufC = 2, kBufAt = 3, kBufBt = 4, kBufCt = 5, kBufAp = 6, kBufBp = 7
};
constexpr int kBufsPerPlan = 8;

// Base pointers: either inline (single plan) or a device table (batch).
struct Ptrs {
  void* p[kBufsPerPlan];
  const uint64_t* table;  // when non-null, buffer id i resolves to table[i]
};

// One chunk of one block for the permute / zero-fill kernel.  The block is an
// n-dimensional array in OUTPUT leg order (dim 0 fastest); element with
// multi-index i sits at src + sum i_d*ss[d] in the source buffer and at
// dst + sum i_d*ds[d] in the destination.  The chunk covers output-linear
// indices start .. start+count-1.  src_buf < 0 means "no source": the value
// is zero (used for coupled charges whose K range is empty).
struct PermTask {
  int64_t src;
  int64_t dst;
  int32_t n;
  int32_t count;
  int32_t start;
  int16_t src_buf;
  int16_t dst_buf;
  float sign;
  // 0: the destination holds the element type; otherwise it is a bf16 hi
  // plane and element x goes in as hi = bf16(x) at dst and
  // lo = bf16(x - hi) at dst + lo (split-BF16x3 operands)
  int32_t lo;
  int32_t dim[kMaxDims];
  int32_t ss[kMaxDims];
  int32_t ds[kMaxDims];
  // division by dim[d] as a multiply-high: for 0 <= x < 2^31,
  // x / dim[d] == (x * mag[d]) >> shr[d]
  uint32_t mag[kMaxDims];
  uint8_t shr[kMaxDims];
};

// One tile of a block permute staged through LDS: the block's source is
// contiguous along one dimension (a) and its destination along another (b).
// The tile covers ea x eb elements (each at most kTileEdge) at a fixed index
// of every other dimension: element (ia, ib) is read at src + ia + ib * sb and
// written at dst + ia * ta + ib (times sign; lo as in PermTask), so the reads
// run along a and the writes along b, both coalesced.
constexpr int kTileEdge = 64;
struct TileTask {
  int64_t src, dst;
  int32_t ea, eb;
  int32_t sb, ta;
  int16_t src_buf, dst_buf;
  float sign;
  int32_t lo;
  int32_t pad_;
};

// One sector GEMM  C~^c (M x N) = A~^c (M x K) * B~^c (K x N), all
// column-major.  mode 0: C~^c is written in place at c (ldc).  mode 1: the
// epilogue scatters every element to its position in C (fused output
// permute) through the row/column maps and the channel-pair table.
// Split-BF16x3 operands (a_buf kBufAp, b_buf kBufBp) are bf16 planes with k
// contiguous: A~ element (m, k) at a + m lda + k, B~ element (k, n) at
// b + n ldb + k, lda = ldb = K rounded up to a multiple of 8 (the padding
// holds zeros), and the lo planes alo and blo elements after the hi planes.
struct GemmDesc {
  int64_t a, b, c;
  int32_t M, N, K;
  int32_t lda, ldb, ldc;
  int32_t a_buf, b_buf, c_buf, mode;  // 32-bit: a 16-bit field read alone is a vector load
  int32_t row_map;    // first entry of this sector in the row map
  int32_t col_map;    // first entry in the column map
  int32_t pair_base;  // first entry in the pair table
  int32_t ncc;        // column channels of this sector (pair = rc * ncc + cc)
  int32_t pad_;
  int64_t alo, blo;   // lo-plane offsets of split operands (elements)
};

// One unit of work of the grouped GEMM: the (m0, n0) tile of sector GEMM
// `gemm` over the K range [k0, k1).  When nsplit > 1 the K range of the tile
// is split over nsplit units; each writes its partial tile to slot
// slot0 + split of the partial buffer, and a second kernel sums the nsplit
// partials of every group in split order (a fixed order, so results do not
// depend on scheduling) and runs the epilogue.
struct GemmTile {
  int32_t gemm;
  int32_t m0;
  int32_t n0;
  int32_t k0;
  int32_t k1;
  int32_t nsplit;
  int32_t split;
  int32_t group;  // index of the split group
  int32_t slot0;  // first partial slot of the split group
  int32_t pad_;
};

// Small-K sector GEMM work as output-stationary block tasks: an output block
// of C (dims/dst strides in C's leg order) whose element i has C~ row
// r = sum i_d rs[d] and column s = sum i_d cs[d] relative to a and b, and value
// sign * sum_k A~[a + r + k lda] B~[b + k + s ldb].
// One range of elements to zero (scaled by beta when beta != 0): elements
// off .. off + len - 1 of buffer `buf`, where len = next range's vstart -
// vstart.  The ranges of a launch are concatenated into one virtual array;
// vstart is where this range starts in it.
struct ZeroRange {
  int64_t off;
  int64_t vstart;
  int32_t buf;
  int32_t pad_;
};
// elements and ranges of one workgroup of the zero-range kernel (at most)
constexpr int kZeroChunk = 8192;
constexpr int kZeroMax = 256;

// Rows or columns of one channel of a small-K sector: first index in the
// sector, count, and the degeneracy of each leg of the channel (the index of
// a row/column within the channel is colex over these, first leg fastest).
struct SkChan {
  int32_t off, count;
  int32_t dim[4];
  // division by dim[l] as a multiply-high (see PermTask)
  uint32_t mag[4];
  uint8_t shr[4];
};

// Rows r0 .. r0 + rows - 1 of one row channel of a sector GEMM with K <= 8,
// against a run of ncols consecutive columns of the sector starting at
// column bcol (which lies at column c0 of column channel cchan; the run
// crosses channels in order).  Output element (row, column) goes to
// pairs[pair + (column channel - cchan)]: base + sum of leg index x stride,
// times the pair's sign.
// Rows of A~ per thread of the row-stationary small-K kernel: several when K
// is small, so that each thread has more loads in flight.
constexpr int smallk_rows_per_thread(int K) { return K <= 2 ? 4 : K <= 4 ? 2 : 1; }

struct SmallKTask {
  int64_t a;  // A~ element of the task's first row, column 0
  int64_t b;  // B~ element of row 0, column 0 of the sector
  int32_t lda, ldb;
  int32_t rows, r0;
  int32_t rchan, cchan, c0, ncols, bcol;
  int32_t pair;
  int16_t nrleg, ncleg;
  int16_t a_buf, b_buf, dst_buf, pad_;
};

// Row (or column) r of a sector of C~: its channel inside the sector and the
// index of each of its legs (up to 4 legs per side, 16 bits each).
struct LegMap {
  int32_t chan;
  int32_t pad_;
  uint16_t idx[4];
};

// Output placement of the channel pair (row channel, column channel) of C~:
// element (r, s) goes to base + sum_l row_idx_l * S[l] + sum_l col_idx_l * S[4+l],
// multiplied by sign.
struct PairDesc {
  int64_t base;
  float sign;
  int32_t pad_;
  int32_t S[8];
};

struct GemmArgs {
  const GemmDesc* descs;
  const GemmTile* tiles;     // tiles grouped by workgroup
  const int32_t* wg_first;   // workgroup w handles tiles wg_first[w] .. wg_first[w+1]-1
  const LegMap* row_map;
  const LegMap* col_map;
  const PairDesc* pairs;
  double* partials;          // split-K partial tiles (tile_m * tile_n each; fp32 values for fp32 accumulators)
  Ptrs ptrs;
  double alpha, beta;
};

// Launchers (tk_kernels.hip).  dtype: 0 fp64, 1 fp32.  precision: tk_precision.
// LDS-staged tiles (one workgroup each), same alpha / beta / split rules
hipError_t launch_permute_tiles(int dtype, const TileTask* tiles, int ntiles, const Ptrs& ptrs, double alpha,
                                double beta, hipStream_t stream, bool split = false);
// split: tasks with lo != 0 write bf16 hi / lo planes (split-BF16x3 operands)
hipError_t launch_permute(int dtype, const PermTask* tasks, const int32_t* wg_first, int nwg,
                          const Ptrs& ptrs, double alpha, double beta, hipStream_t stream, bool split = false);
hipError_t launch_gemm(int dtype, int precision, int tile_m, int tile_n, int tile_k, const GemmArgs& args,
                       int nwg, hipStream_t stream);
hipError_t launch_splitk_reduce(int dtype, int precision, int tile_m, int tile_n, int tile_k, const GemmArgs& args,
                                const GemmTile* groups, int ngroups, hipStream_t stream);
// Elements start .. start + count - 1 of one output block (row channel
// rchan x column channel cchan), or a strip of whole blocks (below), of a
// small-K sector with many columns,
// enumerated in the order of the output's legs (colex, first leg fastest):
// output leg o is leg ((order >> 4o) & 15) of C~ (rows' legs first).  a, b:
// A~ element of the channel's first row, B~ element of its first column.
// nblk > 1: a strip of whole blocks, column channels cchan .. cchan+nblk-1
// of the same row channel (pairs pair .. pair+nblk-1); count is then the
// strip's total (used only to pack workgroups).
struct SkBlockTask {
  int64_t a, b;
  int32_t lda, ldb;
  int32_t rchan, cchan, pair;
  int32_t start, count;
  uint32_t order;
  int16_t nrleg, ncleg, nout;
  int16_t a_buf, b_buf, dst_buf;
  int32_t nblk;
};
hipError_t launch_smallk_blocks(int dtype, int precision, int K, const SkBlockTask* tasks, const int32_t* wg_first,
                                int nwg, const SkChan* chans, const PairDesc* pairs, const Ptrs& ptrs, double alpha,
                                double beta, hipStream_t stream);

// Output runs of the small-K sectors with many columns whose blocks land in
// C directly.  A run is a stretch of consecutive elements of C inside one
// output block, over which the block's linear index (its dimensions in the
// output's leg order, first fastest) also steps by one.
struct SkRun {
  int64_t off;     // first element in the destination buffer
  int64_t vstart;  // first element in the list's concatenation of runs
  int64_t a, b;    // the block's rows in A~ and its first column in B~ (elements)
  int32_t lin0;    // linear index of the run's first element in its block
  int32_t shape;   // the block's dimension record
  int32_t lda;     // A~ stride between consecutive k
  float sign;
  int16_t buf, a_buf, b_buf, pad_;  // destination and operand buffers
  int32_t len;     // elements (host side)
};

// Dimension record of an output block written through runs, shared by all
// blocks with the same extents: its output dimensions of extent above 1 in
// the output's leg order (first fastest), per dimension the division magic
// (floor(x / d) = mulhi(x, mag) >> shift for x < 2^24), the extent, and the
// strides of the leg in A~ and in B~ (one of them 0; the B~ stride counts
// elements, ldb included).  Blocks hold fewer than 2^24 elements and every
// operand offset inside a block, and lda, are below 2^24.
struct SkRunDim {
  uint32_t mag;
  uint32_t dimshr;  // extent | (shift - 32) << 24
  uint32_t sa, sb;
};
struct SkRunShape {
  int32_t nd, pad_[3];
  SkRunDim dim[8];
};
constexpr int kRunChunk = 4096;  // elements of one workgroup
constexpr int kRunMax = 128;     // runs one workgroup touches at most

// Runs of small-K sectors sharing the same K (1..8).  Workgroup w covers
// elements wstart[w] .. wstart[w+1]-1 of the concatenation; first[w] is the
// run holding element wstart[w].
hipError_t launch_smallk_runs(int dtype, int precision, int K, const SkRun* runs, int nruns, const int32_t* first,
                              const int64_t* wstart, int nwg, const SkRunShape* shapes, const Ptrs& ptrs, double alpha,
                              double beta, hipStream_t stream);

// Zero (or beta-scale) the ranges: workgroup w covers virtual elements
// wstart[w] .. wstart[w+1]-1; first[w] is the range holding wstart[w].
hipError_t launch_zero_ranges(int dtype, const ZeroRange* ranges, int nranges, const int32_t* first,
                              const int64_t* wstart, int nwg, const Ptrs& ptrs, double beta, hipStream_t stream);
// Partial trace (Alg. "Abelian Tensor Trace"): one chunk of one output block
// of C, elements start .. start + count - 1 of its linear order over dim
// (first fastest; destination offset sum i_d ds[d]).  Its value is the sum,
// over contributions c0 .. c1 - 1 (the input channels whose free legs give
// this block and whose traced pairs carry equal sectors), of the
// contribution's sign times its sum along the traced diagonal.
struct TraceTask {
  int64_t dst;
  int32_t n, count, start, c0, c1;
  int16_t src_buf, dst_buf;
  int32_t dim[kMaxDims];
  int32_t ds[kMaxDims];
  uint32_t mag[kMaxDims];
  uint8_t shr[kMaxDims];
};
// One input channel feeding an output block: its first element in A, per
// output dimension its stride in A, and per traced pair the degeneracy and
// one diagonal step (the sum of the two legs' strides).
constexpr int kMaxTracePairs = 4;
struct TraceContrib {
  int64_t src;
  double coef;  // the sign of a fermionic trace, a recoupling coefficient
  int32_t nd;
  int32_t ss[kMaxDims];
  int32_t dd[kMaxTracePairs];
  int32_t dstr[kMaxTracePairs];
};
// gather: no contribution has a traced pair (nd == 0 throughout) and the
// contributions of each task share their strides ss, which selects the
// unrolled plain-gather variant.
hipError_t launch_trace(int dtype, const TraceTask* tasks, const int32_t* wg_first, int nwg,
                        const TraceContrib* contribs, const Ptrs& ptrs, double alpha, double beta, bool gather,
                        hipStream_t stream);
// Singular value decomposition of one coupled-sector matrix (R x C,
// column-major) by one-sided Jacobi rotations on its m x n working copy W
// (the matrix, or its transpose when R < C, so that m >= n), with the
// rotations accumulated in V (n x n).  At the end sigma[j] = |W_j| and W_j is
// normalised (the left singular vectors of the working matrix).
struct SvdSector {
  int64_t x;         // the matrix in its buffer
  int64_t w, v, s;   // W, V and sigma in the workspace (elements)
  int32_t R, C, m, n, trans, pad_;
};
constexpr int kSvdThreads = 1024;
// Block Jacobi: columns per block, threads of a block-pair workgroup (one
// 16-thread group per column pair of a round of 2 kSvdBlock columns).
constexpr int kSvdBlock = 16;
constexpr int kSvdRoundThreads = kSvdBlock * 16;
// One block pair of one sector in a round: columns p0 .. p0+np-1 and
// q0 .. q0+nq-1 of its W (nq = 0: a block paired with the empty one).
struct SvdItem {
  int32_t sec, p0, np, q0, nq, pad_;
};
hipError_t launch_svd_init(const SvdSector* secs, int nsec, const double* X, double* ws, hipStream_t stream);
hipError_t launch_svd_round(const SvdItem* items, int nitems, const SvdSector* secs, double* ws, const int32_t* prev,
                            int32_t* flag, int sweep, double tol, hipStream_t stream);
hipError_t launch_svd_finish(const SvdSector* secs, int nsec, double* ws, hipStream_t stream);

// Bytes of the per-device scratch array that the allocation-free
// contraction lays its tables and workspaces into (TK_SCRATCH_BYTES).
constexpr size_t kScratchBytes = size_t(64) << 20;
// Device address of that array on the current device (hipGetSymbolAddress;
// call once per device, with the device current).
hipError_t scratch_address(void** out);

// Small-K sector GEMM tasks that all share the same K (1..8): one
// workgroup per task.
hipError_t launch_smallk(int dtype, int precision, int K, const SmallKTask* tasks, int ntasks, const SkChan* chans,
                         const PairDesc* pairs, const Ptrs& ptrs, double alpha, double beta, hipStream_t stream);
bool gemm_tile_supported(int dtype, int precision, int tile_m, int tile_n, int tile_k);
// Workgroups of the grouped GEMM a CU holds at once for this configuration
// (registers and LDS); the persistent grid is this many per CU.
int gemm_blocks_per_cu(int dtype, int precision, int tile_m, int tile_n, int tile_k);
int num_tile_shapes();
void tile_shape(int i, int* tm, int* tn, int* tk);

}  // namespace tk
