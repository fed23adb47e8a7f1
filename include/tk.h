/*
 * tk.h -- C-ABI of the symmetric-TensorMap contraction library (gfx950).
 *
 * A TensorMap  t : W_1 (x) .. (x) W_N2 -> V_1 (x) .. (x) V_N1  over graded
 * spaces of an abelian symmetry is stored as one dense column-major matrix
 * per coupled charge c (the block-diagonal matrix form of the abelian
 * grouping isomorphism, eq. abeliangrouping).  The library implements
 *   - tk_tensor_permute : Alg. "Abelian Tensor Permutation" (with the
 *                         fermionic exchange sign for U(1) x fZ2 / fZ2),
 *   - tk_tensor_contract: Alg. "Abelian tensor contraction" (permute A,
 *                         permute B, one GEMM per coupled charge, zero block
 *                         for an empty K range, permute C fused into the
 *                         GEMM epilogue),
 *   - tk_tensor_adjoint : blockwise Hermitian conjugate (section "Adjoint").
 * All numerical work runs in hand-written HIP kernels on the device; the host
 * side only plans (block structure, index maps, signs, schedules).
 *
 * Conventions
 * -----------
 * Legs are 0-based (the paper counts from 1) and numbered codomain first,
 * then domain: legs 0..N1-1 are V_1..V_N1, legs N1..N1+N2-1 are W_1..W_N2.
 * A permutation (p, q) takes the p_i-th space of (V_1.., W_1*..) into the
 * new codomain and the q_j-th space of (V_1*.., W_1..) into the new domain
 * (Alg. "Tensor Permute"): a leg that crosses between codomain and domain
 * has its space dualised.
 *
 * Spaces.  tk_space lists the sectors of the underlying space and a dual
 * flag.  `charges` holds nsect * ncomp int32 values, ncomp = 0 for Z1,
 * 1 for Z2 / FZ2 (parity 0 or 1) and U1 (charge), 2 for U1xFZ2 (charge,
 * parity).  A leg on a dual space carries the conjugate charge (-q, same
 * parity) for block keys and charge conservation.  Sectors of one space must
 * be distinct; degeneracies must be >= 1.
 *
 * Storage layout (the "arbitrary but fixed" channel order of the grouping
 * isomorphism, fixed here): coupled charges that occur on both sides are
 * stored in ascending (charge, parity) order, each as an R_c x C_c
 * column-major matrix; rows are the codomain channels (tuples of sector
 * indices) enumerated with the first leg fastest, columns the domain
 * channels likewise; inside a channel block the entries follow
 * eq. linearindex (first index fastest).  tk_tensor_blocks reports every
 * channel with its offset so callers never need to recompute this.
 *
 * Fermions (FZ2, U1xFZ2) follow the graph convention of the section
 * "Fermions and fusion categories" (twist pushed into the right
 * evaluation): a TensorMap is read as a tensor in
 * V_1..V_N1 (x) W*_N2..W*_1 with unchanged coefficients; a permute
 * multiplies a channel by (-1)^{|x||y|} for every pair of legs whose order
 * in that reading is exchanged (R^{JJ}_I = -1); a composition multiplies by
 * (-1)^{|k|} for every contracted leg whose space in the codomain of the
 * right operand is a dual space.
 *
 * Ownership.  All handles are opaque and destroyed by the caller.  A tensor
 * either owns device memory allocated by the library (device_buf == NULL) or
 * wraps caller memory (e.g. a torch tensor's data_ptr) that must outlive the
 * handle and is never freed by the library.  Plans and batches own their
 * device tables and workspaces, all allocated when they are created, so
 * their launches allocate nothing and can be captured in a HIP graph.
 *
 * Asynchrony.  Device work is enqueued on the hipStream_t passed as
 * `stream` (NULL = the null stream) and is not synchronised; the caller
 * orders it.  Host-side planning is thread safe; a plan or batch must not be
 * executed concurrently with itself.
 *
 * Errors.  Every call returns a tk_status; on error the out-parameters are
 * untouched and tk_last_error() returns a thread-local message.  No C++
 * exception crosses this interface.
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tk_status;
#define TK_OK 0
#define TK_ERR_INVALID_ARG 1    /* bad pointer, size, index list or permutation */
#define TK_ERR_SPACE_MISMATCH 2 /* domain(A~) != codomain(B~), or C's spaces wrong */
#define TK_ERR_CHARGE 3         /* sector invalid for the symmetry / repeated */
#define TK_ERR_DTYPE 4          /* dtype or precision combination not allowed */
#define TK_ERR_UNSUPPORTED 5    /* beyond a documented limit (rank, sectors) */
#define TK_ERR_OOM 6            /* device or host allocation failed */
#define TK_ERR_HIP 7            /* a HIP runtime call or kernel launch failed */

typedef enum tk_symmetry {
  TK_SYM_Z1 = 0,     /* no symmetry: one trivial sector per space */
  TK_SYM_Z2 = 1,     /* bosonic Z2 */
  TK_SYM_FZ2 = 2,    /* fermion parity (SVect) */
  TK_SYM_U1 = 3,     /* U(1) */
  TK_SYM_U1_FZ2 = 4  /* U(1) x fZ2 (Deligne product) */
} tk_symmetry;

typedef enum tk_dtype { TK_F64 = 0, TK_F32 = 1 } tk_dtype;

typedef enum tk_precision {
  TK_PREC_NATIVE = 0, /* fp64 MFMA for fp64 tensors, fp32 MFMA for fp32 tensors */
  TK_PREC_F32 = 1,    /* operands rounded to fp32, fp32 MFMA, fp32 accumulation */
  TK_PREC_BF16X3 = 2  /* a = hi + lo (two bf16), hi*hi + hi*lo + lo*hi, fp32 accumulation */
} tk_precision;

typedef struct tk_space {
  int32_t nsect;               /* number of sectors, >= 1 */
  const int32_t* charges;      /* nsect * ncomp values (may be NULL when ncomp == 0) */
  const int64_t* degeneracies; /* nsect values, each >= 1 */
  int32_t isdual;              /* 0: V, 1: V* */
} tk_space;

/* Limits: at most TK_MAX_LEGS legs per side and TK_MAX_RANK in total; at
 * most 255 sectors per space. */
#define TK_MAX_LEGS 8
#define TK_MAX_RANK 8

typedef struct tk_context tk_context;
typedef struct tk_tensor tk_tensor;
typedef struct tk_plan tk_plan;
typedef struct tk_batch tk_batch;
typedef struct tk_svd tk_svd;

/* ---- context ------------------------------------------------------------
 * A context binds a HIP device and owns the plan cache used by
 * tk_tensor_permute / tk_tensor_contract.  tk_context_create makes `device`
 * current on the calling thread. */
tk_status tk_context_create(int32_t device, tk_context** out);
tk_status tk_context_destroy(tk_context* ctx);

/* ---- tensors --------------------------------------------------------------
 * Creates a TensorMap  dom[0] (x)..(x) dom[ndom-1] -> cod[0] (x)..(x) cod[ncod-1].
 * ctx == NULL creates a structure-only handle (no data; usable for queries
 * and planning, not for execution; device_buf must then be NULL).
 * device_buf == NULL: the library allocates (uninitialised) device memory.
 * Otherwise device_buf must hold at least nelem * sizeof(dtype) bytes
 * (buf_bytes) and stay valid while the handle lives. */
tk_status tk_tensor_create(tk_context* ctx, int32_t sym, int32_t dtype, const tk_space* cod,
                           int32_t ncod, const tk_space* dom, int32_t ndom, void* device_buf,
                           uint64_t buf_bytes, tk_tensor** out);
tk_status tk_tensor_destroy(tk_tensor* t);

/* Number of codomain/domain legs, stored elements, fusion channels and
 * coupled charges (any out-pointer may be NULL). */
tk_status tk_tensor_info(const tk_tensor* t, int32_t* sym, int32_t* dtype, int32_t* ncod,
                         int32_t* ndom, int64_t* nelem, int64_t* nblocks, int64_t* nsectors);

/* Channels first..first+count-1 in storage order (coupled charge ascending,
 * then domain channel, then codomain channel).  sector_idx receives
 * count * (ncod + ndom) sector indices (position of each leg's sector in its
 * space's list), offsets the element offset of the block's first entry,
 * ld the leading dimension R_c of its coupled-charge matrix.  Any output
 * pointer may be NULL. */
tk_status tk_tensor_blocks(const tk_tensor* t, int64_t first, int64_t count, int32_t* sector_idx,
                           int64_t* offsets, int64_t* ld);

/* Coupled charges first..first+count-1: charges (count * ncomp), rows R_c,
 * cols C_c and element offset of each matrix. */
tk_status tk_tensor_sectors(const tk_tensor* t, int64_t first, int64_t count, int32_t* charges,
                            int64_t* rows, int64_t* cols, int64_t* offsets);

/* Space of leg `leg` (0-based over codomain then domain).  The returned
 * arrays are owned by the tensor and valid while it lives. */
tk_status tk_tensor_space(const tk_tensor* t, int32_t leg, tk_space* out);

/* Device pointer and size in bytes of the tensor's storage. */
tk_status tk_tensor_data(const tk_tensor* t, void** device_ptr, uint64_t* bytes);

/* ---- spaces of results -----------------------------------------------------
 * Create the (data-holding if ctx != NULL) tensor that tk_tensor_permute,
 * tk_tensor_contract or tk_tensor_adjoint write, with the spaces the
 * algorithms assign.  Buffer arguments as for tk_tensor_create. */
tk_status tk_tensor_create_permuted(tk_context* ctx, const tk_tensor* A, const int32_t* p,
                                    int32_t np, const int32_t* q, int32_t nq, void* device_buf,
                                    uint64_t buf_bytes, tk_tensor** out);
tk_status tk_tensor_create_contracted(tk_context* ctx, const tk_tensor* A, const int32_t* pA,
                                      int32_t npA, const int32_t* qA, int32_t nqA,
                                      const tk_tensor* B, const int32_t* pB, int32_t npB,
                                      const int32_t* qB, int32_t nqB, const int32_t* pAB,
                                      int32_t npAB, const int32_t* qAB, int32_t nqAB,
                                      void* device_buf, uint64_t buf_bytes, tk_tensor** out);
tk_status tk_tensor_create_adjoint(tk_context* ctx, const tk_tensor* A, void* device_buf,
                                   uint64_t buf_bytes, tk_tensor** out);
/* Truncated singular value decomposition, Alg. "Abelian tensor
 * decomposition": A~ = permute(A, (p, q)) (both sides non-empty) is split
 * as U o S o Vh with U : cod(A~) <- W, S : W <- W diagonal and non-negative
 * (descending within each coupled charge), Vh : W <- dom(A~), where the
 * bond space W has one sector per coupled charge of A~, of degeneracy the
 * number of singular values kept there.  Each coupled-charge matrix is
 * decomposed on the device by one-sided Jacobi rotations, as a block method
 * (column blocks of 16; every block pair of every matrix in a round is one
 * workgroup, which rotates its 32 columns by one Jacobi sweep over their
 * Gram matrix); the kept values
 * are the largest over all charges, at most max_dim of them (max_dim < 0:
 * no bound) and only those above cutoff.  Three steps:
 *   tk_svd_create -- enqueues the decomposition on `stream`, waits for it,
 *     and chooses the kept values (TK_ERR_DTYPE unless A is fp64;
 *     TK_ERR_INVALID_ARG if nothing would be kept);
 *   tk_svd_create_factor -- a tensor with the spaces of U (which = 0),
 *     S (1) or Vh (2), on caller storage as tk_tensor_create;
 *   tk_svd_finish -- fills U, S and Vh (waits for the copies) and returns
 *     the truncation error (the norm of the discarded singular values).
 * Sweeps (one pass over all block pairs; the host waits after each) stop
 * when one rotates no pair (a pair counts as orthogonal when
 * |w_p . w_q| <= max(4, sqrt(m)) eps |w_p| |w_q|, m the longer side of the
 * sector matrix: the rounding level of an m-term inner product); a sector
 * still rotating after 60
 * sweeps fails tk_svd_create with TK_ERR_UNSUPPORTED (its values would not
 * be converged).  tk_svd_info reports the number of decomposed sector
 * matrices, of kept values, and the largest sweep count (any pointer may be
 * NULL).
 * The handle owns device workspace until tk_svd_destroy; it allocates, so
 * it is not for graph capture. */
tk_status tk_svd_create(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np,
                        const int32_t* q, int32_t nq, int64_t max_dim, double cutoff, void* stream,
                        tk_svd** out);
tk_status tk_svd_create_factor(tk_context* ctx, const tk_svd* svd, int32_t which, void* device_buf,
                               uint64_t buf_bytes, tk_tensor** out);
tk_status tk_svd_finish(tk_svd* svd, tk_tensor* U, tk_tensor* S, tk_tensor* Vh, double* trunc_err,
                        void* stream);
tk_status tk_svd_info(const tk_svd* svd, int64_t* nsectors, int64_t* nkept, int32_t* max_sweeps);
tk_status tk_svd_destroy(tk_svd* svd);

/* A tensor shaped as the partial trace of A (see tk_tensor_trace). */
tk_status tk_tensor_create_traced(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np,
                                  const int32_t* q, int32_t nq, const int32_t* t1, const int32_t* t2,
                                  int32_t nt, void* device_buf, uint64_t buf_bytes, tk_tensor** out);

/* ---- operations ------------------------------------------------------------
 * C = permute(A, (p, q)).  C must have the permuted spaces and A's dtype. */
tk_status tk_tensor_permute(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np,
                            const int32_t* q, int32_t nq, tk_tensor* C, void* stream);

/* Partial trace, Alg. "Abelian Tensor Trace": C = alpha * tr(A) + beta * C,
 * where legs t1[i] and t2[i] of A (nt pairs, 1..4) are closed with each
 * other and the remaining legs form C's codomain (p) and domain (q), each
 * indexing A's legs (0-based, codomain then domain); p, q, t1 and t2 list
 * every leg of A exactly once.  A traced pair must carry the same sectors
 * and degeneracies and be a vector / co-vector pair in A's bra-ket reading
 * (a codomain leg over V with a domain leg over V, or two codomain legs over
 * V and V*, ...); the trace is diagonal in the sector and in the index.
 * C's spaces are those of tk_tensor_create_traced (the free legs placed as
 * by tk_tensor_permute).  Fermionic symmetries use the graph semantics of
 * the section on fermions (twist pushed into the right evaluation): a
 * channel's sign is the Koszul sign of reordering A's legs so that every
 * traced pair is adjacent with its dual leg first, followed by C's legs.
 * Errors: TK_ERR_INVALID_ARG (bad lists, null or aliased tensors),
 * TK_ERR_SPACE_MISMATCH (pair spaces, C's spaces), TK_ERR_DTYPE,
 * TK_ERR_UNSUPPORTED (more than 4 pairs, strides beyond 32 bits). A and C
 * are caller-owned; the plan is cached in the context; the launch is
 * enqueued on `stream`. */
tk_status tk_tensor_trace(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np,
                          const int32_t* q, int32_t nq, const int32_t* t1, const int32_t* t2, int32_t nt,
                          double alpha, double beta, tk_tensor* C, void* stream);

/* C = alpha * permute(permute(A,(pA,qA)) o permute(B,(pB,qB)), (pAB,qAB)) + beta * C.
 * (pA, qA): free legs of A (codomain of A~) and contracted legs (domain of
 * A~); (pB, qB): contracted legs of B in the same order as qA (codomain of
 * B~) and free legs (domain of B~); (pAB, qAB) index the legs of
 * C~ = A~ o B~, numbered pA-legs then qB-legs.  Requires
 * domain(A~) == codomain(B~) as spaces (sectors, degeneracies, dual flags).
 * A coupled charge of C~ whose K range is empty yields zeros (times alpha).
 * beta == 0 never reads C.  A, B and C must not alias. */
tk_status tk_tensor_contract(tk_context* ctx, const tk_tensor* A, const int32_t* pA, int32_t npA,
                             const int32_t* qA, int32_t nqA, const tk_tensor* B,
                             const int32_t* pB, int32_t npB, const int32_t* qB, int32_t nqB,
                             const int32_t* pAB, int32_t npAB, const int32_t* qAB, int32_t nqAB,
                             double alpha, double beta, int32_t precision, tk_tensor* C,
                             void* stream);

/* The same contraction as tk_tensor_contract, for callers that cannot
 * allocate device memory (code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It calls no hipMalloc or hipFree and no
 * allocating library routine: the plan is rebuilt on the host each call and
 * its device tables and workspaces (the permuted operands A~ and B~, C~ when
 * the output permute runs after the GEMM, split-K partial tiles) are laid
 * into one per-device scratch array of TK_SCRATCH_BYTES, which the library's
 * code object holds on every device it runs on until the process ends (its
 * address is looked up once per device, when the first context on that
 * device is created).  The tables reach the array by one asynchronous copy
 * on `stream`, then the kernels of tk_tensor_contract run on `stream` with
 * the same schedule, so the result is bitwise the same.  Contractions whose
 * tables and workspaces exceed TK_SCRATCH_BYTES fail with
 * TK_ERR_UNSUPPORTED (nothing is enqueued).  Every call on one device uses
 * the same array and leaves its contents behind: calls on one stream are
 * ordered, but calls that overlap on one device (two streams, or two host
 * threads with different streams) race on the array and give wrong results.
 * The host side of calls on one device is serialised internally. */
#define TK_SCRATCH_BYTES (64ull << 20)
tk_status tk_tensor_contract_noalloc(tk_context* ctx, const tk_tensor* A, const int32_t* pA, int32_t npA,
                                     const int32_t* qA, int32_t nqA, const tk_tensor* B, const int32_t* pB,
                                     int32_t npB, const int32_t* qB, int32_t nqB, const int32_t* pAB, int32_t npAB,
                                     const int32_t* qAB, int32_t nqAB, double alpha, double beta, int32_t precision,
                                     tk_tensor* C, void* stream);
/* Number of device allocations the library has made in this process
 * (tensors created without a buffer, plan and batch tables, workspaces). */
uint64_t tk_device_alloc_count(void);

/* C = A^dagger: codomain and domain exchange, every coupled-charge matrix is
 * transposed (conjugation is the identity on real data). */
tk_status tk_tensor_adjoint(tk_context* ctx, const tk_tensor* A, tk_tensor* C, void* stream);

/* ---- plans -----------------------------------------------------------------
 * A plan fixes everything structural about one contraction (tensors may be
 * structure-only) and owns its device tables and workspaces.  Executing it
 * on data-holding tensors with the same structures enqueues: the operand
 * permutes (one launch), the grouped sector GEMM with the output permute
 * fused into its epilogue (one persistent launch), and zero blocks for empty
 * K ranges. */
tk_status tk_plan_contract(tk_context* ctx, const tk_tensor* A, const int32_t* pA, int32_t npA,
                           const int32_t* qA, int32_t nqA, const tk_tensor* B, const int32_t* pB,
                           int32_t npB, const int32_t* qB, int32_t nqB, const int32_t* pAB,
                           int32_t npAB, const int32_t* qAB, int32_t nqAB, int32_t precision,
                           const tk_tensor* C, tk_plan** out);
tk_status tk_plan_execute(tk_plan* plan, const tk_tensor* A, const tk_tensor* B, tk_tensor* C,
                          double alpha, double beta, void* stream);
tk_status tk_plan_destroy(tk_plan* plan);

/* Enqueue only some stages of a plan, in the fixed order operand permutes
 * (TK_STAGE_PERMUTE), grouped GEMM (TK_STAGE_GEMM), zero blocks
 * (TK_STAGE_ZERO); executing all three equals tk_plan_execute.  Lets a
 * caller bracket one stage with events (per-kernel timing).
 * TK_STAGE_PERMUTE_A and TK_STAGE_PERMUTE_B are the operand permute of A
 * alone and of B alone (with TK_PREC_BF16X3: that operand's bf16 planes);
 * the two together equal TK_STAGE_PERMUTE, which runs both in one launch.
 * They let a caller enqueue the permute of an operand that is ready early
 * (an input of a chain of contractions) on another stream, concurrently
 * with earlier work, and the rest of the plan after an event.  The GEMM
 * stage needs both permutes done; the zero stage of a plan whose output is
 * permuted after the GEMM (see tk_plan_counts) needs the GEMM stage done. */
#define TK_STAGE_PERMUTE 1
#define TK_STAGE_GEMM 2
#define TK_STAGE_ZERO 4
#define TK_STAGE_ALL 7
#define TK_STAGE_PERMUTE_A 8
#define TK_STAGE_PERMUTE_B 16
tk_status tk_plan_execute_stages(tk_plan* plan, const tk_tensor* A, const tk_tensor* B, tk_tensor* C,
                                 double alpha, double beta, int32_t stages, void* stream);

/* Plan statistics: number of sector GEMMs with K > 0 (MFMA or streamed), useful block flops
 * (sum of 2 M N K), number of zero-filled coupled charges, workspace bytes,
 * and the GEMM tile configuration in use (any pointer may be NULL). */
tk_status tk_plan_info(const tk_plan* plan, int64_t* ngemm, double* flops, int64_t* nzero,
                       int64_t* workspace_bytes, int32_t* tile_m, int32_t* tile_n, int32_t* tile_k);
/* Work-list sizes of a plan, 14 values: operand-permute tasks and
 * workgroups, zero-block tasks and workgroups, small-K row / block tasks and
 * their workgroups, MFMA GEMM descriptors, tiles (work units), workgroups,
 * split-K groups, split-K partial slots, the schedule's estimated makespan
 * in 16-deep stages (rounded), and small-K output runs and their
 * workgroups. */
tk_status tk_plan_counts(const tk_plan* plan, int64_t* counts /* 14 values */);

/* (M, N, K) of sector GEMMs first..first+count-1 (3 * count values). */
tk_status tk_plan_gemms(const tk_plan* plan, int64_t first, int64_t count, int64_t* mnk);

/* Host copies of a plan's work lists for the kernels that stage a
 * workgroup's items in LDS: kind = 0 the zero ranges (empty-K blocks that
 * are contiguous ranges of C), kind = K (1..8) the output runs of the
 * small-K sectors with that K.  The items of a list are laid end to end;
 * counts receives 3 values: items, workgroups, dimension records (0 for
 * zero ranges).  Every other pointer may be NULL; otherwise it receives, per
 * item, vstart (its first element in the concatenation) and len (elements),
 * and for runs lin0 (linear index of the run's first element in its output
 * block) and shape (its dimension record); first and wstart (workgroups + 1
 * values each): workgroup w covers elements wstart[w] .. wstart[w+1]-1 and
 * item first[w] holds element wstart[w]; dimrec (25 values per record): the
 * number of dimensions nd (<= 8), then per dimension its extent and the
 * magic and shift of the multiply-high division the kernel splits linear
 * indices with (floor(x / extent) = (x * magic) >> shift for x < 2^24).
 * Call once with NULL arrays to size them.  Host only; lets a CPU test
 * replay every LDS index the kernels form. */
tk_status tk_plan_worklist(const tk_plan* plan, int32_t kind, int64_t* counts, int64_t* vstart, int64_t* len,
                           int32_t* lin0, int32_t* shape, int32_t* first, int64_t* wstart, int32_t* dimrec);

/* Channel map of a permute: for every channel i of A (storage order) the
 * channel index of C it lands in and its sign (+1 / -1).  Host only. */
tk_status tk_permute_map(const tk_tensor* A, const int32_t* p, int32_t np, const int32_t* q,
                         int32_t nq, const tk_tensor* C, int64_t* dst_block, int32_t* sign);

/* ---- batches ---------------------------------------------------------------
 * A batch binds n plans to their data-holding tensors and merges them: all
 * operand permutes in one launch, every sector GEMM of every plan in one
 * persistent grouped-GEMM launch (cost-sorted tiles), all zero blocks in one
 * launch.  tk_batch_launch enqueues that sequence; tk_batch_capture records
 * it once into a HIP graph which tk_batch_replay then launches. */
tk_status tk_batch_create(tk_context* ctx, tk_plan* const* plans, const tk_tensor* const* A,
                          const tk_tensor* const* B, tk_tensor* const* C, int32_t n,
                          double alpha, double beta, tk_batch** out);
tk_status tk_batch_launch(tk_batch* batch, void* stream);
tk_status tk_batch_capture(tk_batch* batch, void* stream);
tk_status tk_batch_replay(tk_batch* batch, void* stream);
tk_status tk_batch_info(const tk_batch* batch, int64_t* ngemm, int64_t* ntiles, double* flops,
                        int32_t* tile_m, int32_t* tile_n, int32_t* tile_k);
tk_status tk_batch_destroy(tk_batch* batch);

/* ---- tile configurations --------------------------------------------------
 * Tile configurations the grouped GEMM supports: (tile_m, tile_n, tile_k)
 * triples, tile_k being the K depth staged through LDS per step.
 * tk_plan_set_tile / tk_batch_set_tile choose one (re-scheduling the tiles,
 * which drops a captured graph); the autotuner in the Python package times
 * the candidates and persists the winner per shape class. */
tk_status tk_tile_shapes(int32_t* count, int32_t* tile_mnk /* 3 * count, may be NULL */);
tk_status tk_plan_set_tile(tk_plan* plan, int32_t tile_m, int32_t tile_n, int32_t tile_k);
tk_status tk_batch_set_tile(tk_batch* batch, int32_t tile_m, int32_t tile_n, int32_t tile_k);

/* ---- SU(2): leg permutations by recoupling ---------------------------------
 * Section "Non-abelian symmetries" (fusion trees, the canonical expansion of
 * a tensor map over fusion-splitting tree pairs) and Alg. "Non-abelian
 * Tensor Transformation": each reduced array of the output is a sum of
 * coefficient * permuted input reduced arrays; the coefficients are
 * products of F-moves (6j symbols) and R-moves (exchange phases) of the
 * Section "Fusion Tree Manipulations", computed on the host when the plan
 * is made.
 *
 * Legs: n1 codomain legs then n2 domain legs (n1, n2 >= 1, n1 + n2 <= 8).
 * Leg l has nsec[l] sectors (1..64); twoj and deg list all sectors of all
 * legs in leg order: twice the spin (0..64, strictly ascending within a leg)
 * and the degeneracy (>= 1).  A splitting tree of legs a_1..a_N is the
 * canonical left-to-right tree: e_1 = a_1, e_k in e_{k-1} x a_k, e_N = c
 * (Condon-Shortley Clebsch-Gordan vertices); domain trees are adjoints of
 * splitting trees of the domain legs.
 *
 * Storage (input and output alike): one column-major matrix per coupled
 * spin c, ascending c, only spins with both rows and columns, laid end to
 * end.  Rows are the codomain trees of c, columns the domain trees of c;
 * a tree takes prod(deg) consecutive rows (columns), its first leg fastest.
 * The trees of one c are ordered by outer sectors (colex, first leg
 * fastest), then by intermediates e_2..e_{N-1} (colex, e_2 fastest).
 *
 * permute(A, (p, q)): output codomain leg k is input leg p[k], output
 * domain leg k is input leg q[k]; (p, q) lists every input leg once.  Legs
 * may move between codomain and domain (the transposes and general
 * permutes of the section on index manipulations): a leg that changes
 * sides carries the dual of its space.  A leg over a dual space keeps the
 * spins of its sectors (SU(2) irreps are self-dual) and its canonical trees
 * carry the isomorphism Z between V_j* and V_j on the outer line (section
 * "Duality Fusion Tree Manipulations"), here Z mapping the dual basis
 * vector of m to (-1)^(j-m) times the vector of -m.  Coefficients of braids
 * within each side come from F- and R-moves; when a leg crosses (or a leg is
 * dual) each coefficient is the overlap of the output tree pair with the
 * input tree pair with its legs reordered, summed over magnetic quantum
 * numbers with Clebsch-Gordan vertices (bends act on components as the
 * identity, pairing a basis with its dual basis).
 *
 * tk_su2_plan_create: builds both structures and the coefficient table on
 *   the host and copies the device tables to the current HIP device (the
 *   plan is bound to it; with no device present the plan is host only:
 *   its queries work, tk_su2_permute refuses it); the caller owns *out
 *   (tk_su2_plan_destroy).
 *   Errors: TK_ERR_INVALID_ARG (null pointers, leg counts, bad p or q,
 *   degeneracies), TK_ERR_CHARGE (spins), TK_ERR_UNSUPPORTED (more than 8
 *   legs, a reduced array beyond 2^31 elements, strides beyond 32 bits).
 * tk_su2_plan_info: element counts of the input and output storage and the
 *   number of (output pair, input pair) contributions (any may be null).
 * tk_su2_plan_contribs: copies the host table, one entry per contribution:
 *   first element of the output reduced array, first element of the input
 *   reduced array, coefficient; cap >= the contribution count.
 * tk_su2_permute: C = alpha * permute(A, (p, q)) + beta * C on `stream`;
 *   A and C are device arrays of dtype (TK_F64 or TK_F32) with the plan's
 *   input and output sizes, caller-owned, not aliased; beta == 0 never
 *   reads C.  The current device must be the plan's (TK_ERR_INVALID_ARG
 *   otherwise).  One launch that allocates nothing, so it may be captured
 *   in a HIP graph; calls with one plan may overlap (the plan is only
 *   read).  The plan must outlive the work enqueued with it. */
typedef struct tk_su2_plan tk_su2_plan;
tk_status tk_su2_plan_create(int32_t n1, int32_t n2, const int32_t* nsec, const int32_t* twoj, const int64_t* deg,
                             const int32_t* p, const int32_t* q, tk_su2_plan** out);
/* As tk_su2_plan_create, with isdual[l] != 0 for input legs over dual
 * spaces (NULL: none) and an output of np codomain legs p[0..np-1] and nq
 * domain legs q[0..nq-1] (np, nq >= 1, np + nq = n1 + n2).
 * tk_su2_plan_create(n1, n2, .., p, q, out) is this call with isdual NULL,
 * np = n1 and nq = n2. */
tk_status tk_su2_plan_create_dual(int32_t n1, int32_t n2, const int32_t* nsec, const int32_t* twoj,
                                  const int64_t* deg, const int32_t* isdual, const int32_t* p, int32_t np,
                                  const int32_t* q, int32_t nq, tk_su2_plan** out);
/* The output's leg counts and, per output leg, whether it is over a dual
 * space (n1 + n2 values; any pointer may be NULL).  Host only. */
tk_status tk_su2_plan_legs(const tk_su2_plan* plan, int32_t* n1, int32_t* n2, int32_t* isdual);
tk_status tk_su2_plan_info(const tk_su2_plan* plan, int64_t* in_size, int64_t* out_size, int64_t* ncontrib);
tk_status tk_su2_plan_contribs(const tk_su2_plan* plan, int64_t cap, int64_t* dst, int64_t* src, double* coef);
tk_status tk_su2_permute(tk_su2_plan* plan, int32_t dtype, const void* A, void* C, double alpha, double beta,
                         void* stream);
tk_status tk_su2_plan_destroy(tk_su2_plan* plan);

/* ---- misc ------------------------------------------------------------------ */
const char* tk_last_error(void);
const char* tk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TK_H */
