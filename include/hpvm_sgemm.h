/*
 * hpvm_sgemm.h -- C ABI of the MI355X (gfx950) lowering of the HPVM sgemm
 * dataflow graph (HPVM technical report, arXiv:1611.00860).
 *
 * The graph (Sec. 6.1, listing "SGEMM in HPVM"; drawing in Fig. "Dataflow
 * graph of sgemm") has a single-instance root node SgemmRoot, a 2-D grid of
 * SgemmInternal instances, and inside each of them an Allocation leaf and a
 * 2-D grid of SgemmLeaf instances.  Sec. 3.4 lowers that hierarchy onto a GPU
 * as tiles: leaf instances form one tile (a workgroup), the parent's
 * instances form the grid of tiles, and memory the Allocation node obtains
 * with llvm.hpvm.malloc lives in the scratchpad.  This library is that
 * lowering written by hand for CDNA4:
 *
 *   SgemmRoot          -> one kernel launch (hpvm_sgemm, hpvm_launch_root)
 *   SgemmInternal grid -> workgroups, one per tile_m x tile_n block of C
 *   SgemmLeaf grid     -> lanes; in the MFMA lowerings each wavefront owns a
 *                         leaf_m x leaf_n sub-tile held as MFMA accumulators
 *   Allocation         -> LDS, sized on the host before the launch (the
 *                         backend's rewritten Allocation1 of Sec. 6.3)
 *
 * Storage: every matrix is row-major.  A is m x k with leading dimension
 * lda >= k, B is k x n with ldb >= n, C is m x n with ldc >= n.  All device
 * pointers are owned by the caller; the library never allocates, frees or
 * copies them (the paper's runtime free calls are no-ops as well, Sec. 6.3).
 * C is updated in place: A and B are `in`, C is `in out` (Sec. 2.3).
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Every launch is asynchronous on that stream, like the paper's
 * llvm.hpvm.launch (Table 1); hpvm_wait is its llvm.hpvm.wait.
 *
 * Errors: every entry point returns an hpvm_status.  Argument checks run in
 * argument order before any HIP call, so a rejected call touches no device
 * state; hpvm_last_error() then names the first offending argument.  No C++
 * exception crosses this interface.  The library keeps no per-call state
 * other than a thread-local error message and the explicit plan / graph
 * handles below.
 */
#ifndef HPVM_SGEMM_H
#define HPVM_SGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
typedef enum hpvm_status {
  HPVM_OK = 0,
  HPVM_INVALID_ARG = -1,      /* a size, leading dimension or pointer is bad */
  HPVM_UNSUPPORTED = -2,      /* tile not in the compiled menu, misalignment */
  HPVM_HIP_ERROR = -3,        /* the HIP runtime reported an error           */
  HPVM_WORKSPACE_TOO_SMALL = -4,
  HPVM_BAD_HANDLE = -5,       /* plan, graph or stream handle unknown/closed */
  HPVM_QUEUE_FULL = -6,       /* stream: every slot holds an unpopped item   */
  HPVM_TIMEOUT = -7,          /* a bounded wait ran out; the call may be     */
                              /* repeated                                    */
  HPVM_STREAM_ENDED = -8      /* the streaming kernel has exited             */
} hpvm_status;

/* ---- arithmetic of the bulk products ------------------------------------ */
/* The paper's sgemm is single precision throughout (Sec. 5.1).  The two other
 * precisions keep FP32 storage and FP32 accumulation and change only the
 * product operands:
 *   HPVM_PREC_BF16   : A and B rounded to bfloat16 (nearest-even) on load.
 *   HPVM_PREC_BF16X3 : each element split as hi = bf16(x), lo = bf16(x - hi);
 *                      the product uses hi*hi + hi*lo + lo*hi.              */
typedef enum hpvm_precision {
  HPVM_PREC_FP32 = 0,
  HPVM_PREC_BF16 = 1,
  HPVM_PREC_BF16X3 = 2
} hpvm_precision;

/* ---- tile: the shape of the two-level hierarchy ------------------------- */
/* tile_m x tile_n : the block of C one SgemmInternal instance (workgroup)
 *                   owns; grid = ceil(n / tile_n) x ceil(m / tile_m).
 * tile_k          : depth of the K-slab of A and B the Allocation node
 *                   stages in LDS per step.
 * leaf_m x leaf_n : outputs per leaf unit.  1 x 1 selects the literal
 *                   lowering: one lane per SgemmLeaf instance, one output
 *                   each, tile_n x tile_m lanes per workgroup, and an
 *                   Allocation of tile_m * tile_n floats holding a tile_k
 *                   (= tile_m) x tile_n slab of B, as in Sec. 6.1-6.3.
 *                   Larger values select an MFMA lowering in which every
 *                   wavefront owns a leaf_m x leaf_n sub-tile of C.
 * stages          : the Allocation node's LDS stages.  0 with tile_k = 0
 *                   and leaf 1 x 1: no Allocation node and no SgemmInternal
 *                   level -- the untiled one-level graph the paper compares
 *                   tiling against (Sec. 3.4, 5.1): one lane per element of
 *                   C reading A and B from global memory, tile_m x tile_n
 *                   lanes per launch group; 1 = one buffer
 *                   (literal lowering); 2 = two stages filled through
 *                   registers, conversion to bfloat16 (if any) fused into
 *                   that copy; 3 = staged BF16 / bf16x3 lowering: operands
 *                   converted into a workspace by a separate pass, then
 *                   moved into LDS stages: straight from HBM for every BF16
 *                   tile and for bf16x3's 256 x 256 tile and 128 x 128 x 64
 *                   tile with 64 x 32 leaves, through registers for
 *                   bf16x3's others; hpvm_sgemm_ws only.
 *                   DMA-fed tiles: FP32 tiles with leaf_n = 128, and BF16 /
 *                   bf16x3 tiles of 256 x 256 with 64 x 128 or 128 x 128
 *                   leaves or with stages = 4 have a ring of `stages` LDS
 *                   stages filled straight from HBM (BF16: FP32 slabs,
 *                   rounded to bfloat16 as each MFMA fragment is read).
 *                   They run problems with m, n at least the tile, n a
 *                   multiple of 4, k a multiple of tile_k, A, B and C
 *                   16-byte aligned with leading dimensions that are
 *                   multiples of 4 (edge tiles computed from a corner moved
 *                   inward, storing only the outputs they own); any other
 *                   problem given such a tile runs FP32's 128 x 128 x 16
 *                   tile, or the register-staged BF16 / bf16x3 tile of the
 *                   same size with tile_k = 32.
 * hpvm_tile_menu lists the combinations compiled into this library.       */
typedef struct hpvm_tile {
  int32_t tile_m;
  int32_t tile_n;
  int32_t tile_k;
  int32_t leaf_m;
  int32_t leaf_n;
  int32_t stages;
} hpvm_tile;

/* ---- the root node's packed argument block ------------------------------ */
/* Byte-compatible with the paper's %struct.RootIn (Sec. 6.1): packed, 88
 * bytes, fields in this order.  bytesX give the extent of each array in
 * bytes; the grid and block fields are the SgemmInternal and SgemmLeaf
 * instance counts, so m = grid_y * block_y and n = grid_x * block_x (the
 * paper passes no m or n).                                                 */
#pragma pack(push, 1)
typedef struct hpvm_root_in {
  const float* A;
  int64_t bytesA;
  int32_t lda;
  const float* B;
  int64_t bytesB;
  int32_t ldb;
  float* C;
  int64_t bytesC;
  int32_t ldc;
  int32_t k;
  float alpha;
  float beta;
  int32_t block_x;
  int32_t block_y;
  int32_t grid_x;
  int32_t grid_y;
} hpvm_root_in;
#pragma pack(pop)

/* ---- structural description of one lowered graph instance -------------- */
typedef struct hpvm_dfg {
  int32_t root_instances; /* always 1: the root has one dynamic instance   */
  int32_t grid_x;         /* SgemmInternal instances along n (columns)     */
  int32_t grid_y;         /* SgemmInternal instances along m (rows)        */
  int32_t block_x;        /* lanes per workgroup along x                   */
  int32_t block_y;        /* lanes per workgroup along y                   */
  int32_t waves;          /* 64-lane wavefronts per workgroup              */
  int64_t alloc_bytes;    /* LDS bytes the Allocation node provides        */
  int32_t k_slabs;        /* ceil(k / tile_k): trips of the staging loop   */
  int32_t lowering;       /* 0 literal, 1 FP32 MFMA, 2 BF16 MFMA,
                             3 bf16x3 MFMA, 4 staged BF16, 5 staged bf16x3,
                             6 untiled (one-level graph)                   */
  int32_t splits;         /* contraction slices the launch runs (1 = the
                             whole k in one pass; see hpvm_sgemm_ws)       */
  int32_t reserved;       /* 0                                             */
  hpvm_tile tile;         /* the tile the launch uses                      */
} hpvm_dfg;

/* One edge or binding of the static graph (Sec. 2.1, Table 1 createEdge,
 * bind.input).  Nodes: 0 SgemmRoot, 1 SgemmInternal, 2 Allocation,
 * 3 SgemmLeaf.  kind 0 = dataflow edge (src output port -> dst input port),
 * kind 1 = input binding (parent input port -> child input port).          */
typedef struct hpvm_edge {
  int32_t kind;
  int32_t src_node;
  int32_t dst_node;
  int32_t src_port;
  int32_t dst_port;
  int32_t all_to_all; /* edges: 1 all-to-all replication, 0 one-to-one */
} hpvm_edge;

/* ======================================================================== */
/* Single sgemm                                                             */
/* ======================================================================== */

/* C <- alpha * A B + beta * C  (the sgemm node of Sec. 6.1; operand order as
 * SgemmLeaf's with m and n made explicit).
 *   m, n, k      : sizes, >= 0.  m == 0 or n == 0 returns HPVM_OK without a
 *                  launch.  k == 0 or alpha == 0 gives C <- beta * C.
 *   alpha, beta  : scalars.  beta == 0 never reads C (NaN in C is
 *                  overwritten); alpha == 0 never reads A or B.
 *   A, B, C      : device pointers (row-major, see above); may be NULL only
 *                  when the matrix is not read or written.
 *   prec         : hpvm_precision.
 *   tile         : hierarchy shape, or NULL to take the autotuned choice for
 *                  this shape class (until hpvm_autotune has run, the
 *                  built-in default: the menu's entry 0 when it gives at
 *                  least 256 tiles; else the DMA-fed 128 x 128 x 32 tile
 *                  if that does, else FP32 64 x 64 x 16, BF16 and bf16x3
 *                  64 x 64 x 32).  Must be
 *                  in hpvm_tile_menu for prec and not need a workspace
 *                  (stages != 3).
 *   stream       : hipStream_t or NULL.
 * Returns HPVM_OK once the work is enqueued.  The MFMA lowerings use 16-byte
 * vector loads where A, B, C and their leading dimensions allow and scalar
 * loads elsewhere; any alignment is accepted.                              */
int hpvm_sgemm(int64_t m, int64_t n, int64_t k, float alpha, const float* A,
               int64_t lda, const float* B, int64_t ldb, float beta, float* C,
               int64_t ldc, int32_t prec, const hpvm_tile* tile, void* stream);

/* hpvm_sgemm with a workspace: the only way to run the staged BF16 / bf16x3
 * lowering (tiles with stages == 3), which first rewrites A and B as
 * zero-padded bfloat16 planes (B transposed so k is contiguous; hi and lo
 * planes for bf16x3) in `workspace` and then runs a GEMM over them; and
 * the split contraction of the DMA-fed tiles (FP32: leaf_n == 128; BF16 and
 * bf16x3: stages 2 and 4): a whole-tile
 * problem (m, n multiples of the tile, A, B, C 16-byte aligned with leading
 * dimensions that are multiples of 4) whose tiles would not cover 256 CUs
 * runs as s contraction slices (s doubled from 1 while tiles * s < 256, at
 * most 16, each slice a whole number of slabs and at least 256 deep; only
 * when tiles * s reaches 256), each writing an m x n partial sum to
 * `workspace`, then one launch forming C <- alpha * (sum of the partials,
 * in slice order) + beta * C.  Results then differ from the single launch
 * by rounding only.
 * workspace: device memory, 16-byte aligned, at least
 * hpvm_sgemm_workspace_bytes(m, n, k, prec, tile) bytes (may be NULL when
 * that is 0); its contents are scratch.  For a split tile it is
 * optional: NULL or fewer bytes run the single launch.  tile == NULL takes
 * the autotuned overall winner; with no autotuned entry, problems that
 * even 128 x 128 tiles would not cover 256 CUs with (BF16 and bf16x3: with
 * k >= 2048) take the DMA-fed tile with the fewest slices (the first in
 * menu order on a tie) when the workspace holds the partial sums; other
 * BF16 products of at least 2^31 multiply-adds (m n k) take the first
 * staged tile, or 128 x 128 x 64 with 64 x 32 leaves when the first would
 * give fewer than 256 tiles (bf16x3 only when the DMA-fed 256 x 256 tile
 * would not cover the CUs or does not suit k and n), and others
 * hpvm_sgemm's choice.  Every other argument and rule is hpvm_sgemm's.     */
int hpvm_sgemm_ws(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda,
                  const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int32_t prec,
                  const hpvm_tile* tile, void* workspace, int64_t workspace_bytes, void* stream);

/* Workspace bytes hpvm_sgemm_ws needs for these sizes and tile (NULL = the
 * tile it would pick): the staged lowering's planes, or s * m * n * 4 for a
 * split contraction of s slices; 0 otherwise.                              */
int hpvm_sgemm_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t prec,
                               const hpvm_tile* tile, int64_t* bytes);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * hpvm_sgemm_ws with, as its workspace, a fixed array of
 * HPVM_NOALLOC_SCRATCH_BYTES bytes of device memory that the library holds
 * on each device it runs on (from that device's first call until the
 * process ends).  The call allocates and frees nothing.  Arguments, checks,
 * results and errors are hpvm_sgemm_ws's for a workspace of that size: with
 * tile == NULL the choice is the one that workspace allows (a split
 * contraction or the staged BF16 / bf16x3 planes only when they fit); an
 * explicit tile of the staged lowering whose planes need more than
 * HPVM_NOALLOC_SCRATCH_BYTES is refused with HPVM_WORKSPACE_TOO_SMALL
 * before any device work, and an explicit split tile whose partial
 * sums do not fit runs as one launch.  The array of the current device is
 * used, so `stream` must belong to the current device.  Every call on a
 * device shares that device's array: calls that overlap in time on one
 * device (two streams, or two host threads) race on it and must be
 * serialized by the caller; calls on one stream are ordered and safe.      */
#define HPVM_NOALLOC_SCRATCH_BYTES ((int64_t)32 << 20)
int hpvm_sgemm_noalloc(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda,
                       const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int32_t prec,
                       const hpvm_tile* tile, void* stream);

/* The paper's launch of the root node with its packed argument block
 * (Sec. 6.3, LaunchDataflowGraph unpacking the 88-byte block and calling the
 * generated SgemmRoot2).  Uses the literal lowering: block_x x block_y lanes
 * per workgroup, one output each, grid_x x grid_y workgroups, Allocation =
 * block_x * block_y floats of LDS.  Every byte extent is checked against the
 * sizes it implies; block_x * block_y must be a multiple of 64 and at most
 * 1024.                                                                     */
int hpvm_launch_root(const hpvm_root_in* args, void* stream);

/* Completes all work enqueued on `stream` (llvm.hpvm.wait, Table 1) and
 * reports an asynchronous HIP error if one occurred.                       */
int hpvm_wait(void* stream);

/* ======================================================================== */
/* Graph structure queries (host only, no device access)                    */
/* ======================================================================== */

/* The Allocation node: LDS bytes one SgemmInternal instance needs for
 * `tile` at precision `prec`.  For the literal lowering this is
 * (tile_m * tile_n) << 2, the formula of the Allocation node function in
 * Sec. 6.1.                                                                 */
int hpvm_alloc_bytes(const hpvm_tile* tile, int32_t prec, int64_t* bytes);

/* The instance of the sgemm graph (Sec. 6.1) that hpvm_sgemm would launch
 * for these sizes, as lowered by Sec. 3.4 and 6.3: the SgemmInternal grid
 * (grid_x x grid_y workgroups), the SgemmLeaf lanes of one instance, the
 * Allocation node's LDS bytes, the staging-loop trips and the lowering.
 * tile == NULL describes the tile hpvm_sgemm picks (autotuned, else the
 * built-in choice); splits is 1 (hpvm_sgemm never splits the contraction).
 * Host only: reads no device state.                                        */
int hpvm_describe(int64_t m, int64_t n, int64_t k, int32_t prec,
                  const hpvm_tile* tile, hpvm_dfg* out);

/* The same for hpvm_sgemm_ws given a workspace of `workspace_bytes` (>= 0):
 * the tile it picks for tile == NULL with that workspace, and in `splits`
 * the contraction slices it runs (a split tile whose partial sums do
 * not fit runs as one launch, splits = 1).                                 */
int hpvm_describe_ws(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile,
                     int64_t workspace_bytes, hpvm_dfg* out);

/* The static edge and binding table of the sgemm graph.  Writes at most
 * `capacity` entries to `out` (which may be NULL when capacity is 0) and
 * the total count to *count.                                               */
int hpvm_dfg_edges(hpvm_edge* out, int32_t capacity, int32_t* count);

/* Compiled tiles for `prec`: writes at most `capacity` entries, total count
 * to *count.  Entry 0 is the default when no tile is given (see
 * hpvm_sgemm for the exceptions).                                           */
int hpvm_tile_menu(int32_t prec, hpvm_tile* out, int32_t capacity,
                   int32_t* count);

/* ======================================================================== */
/* Backward pass                                                            */
/* ======================================================================== */
/* Gradient of a scalar loss L through C_out = alpha A B + beta C_in, given
 * the upstream gradient G = dL/dC_out (m x n).  The paper defines no
 * backward; these are the closed forms of the same definition:
 *   dA     = alpha G B^T                 (m x k)
 *   dB     = alpha A^T G                 (k x n)
 *   dalpha = sum_ij G_ij (A B)_ij        (= <A, G B^T>, fused into dA's pass)
 *   dbeta  = sum_ij G_ij C_in_ij
 *   dC_in  = beta G                      (zeros when beta == 0: C_out then
 *                                         does not depend on C_in)
 * dA and dB run on an MFMA lowering of `prec` (FP32, BF16 or bf16x3
 * products, FP32 accumulation): the fused one reads B (for dA) and A (for
 * dB) in transposed form; the staged one (tiles with stages == 3) folds
 * that transposition into its conversion passes, and converts G for both
 * products in one pass that also writes dC_in and the partials of dbeta.
 * The first menu entry of FP32 and of BF16 (256 x 256 x 32, leaf 64 x 128)
 * runs both products on the DMA-fed loop with their contractions split into
 * slices (partial sums in the workspace, then one ordered summing pass that
 * also writes dC_in and dbeta's partials); BF16 there rounds the FP32 slabs
 * in the fragment reads, with no conversion pass.  Passes that are not
 * whole, 16-byte aligned tiles take another entry (FP32: per pass; BF16:
 * the whole call takes the staged 128 x 128 x 64 entry).  The built-in
 * choice takes the DMA entry for FP32 only.
 * The two scalars are reduced
 * in FP32 with fixed-order tree sums, so repeated calls give identical bits.
 * Any of dA, dB, dC_in, dalpha, dbeta may be NULL to skip that output.
 * dalpha and dbeta are single device floats.  A, B, C_in and G are device
 * matrices with the row-major layouts of hpvm_sgemm (G and dC_in like C,
 * dA like A, dB like B); C_in is only read when dbeta is requested.
 * tile: an entry of hpvm_sgemm_backward_menu(prec), or NULL for the
 * hpvm_autotune_backward choice for these sizes (else a built-in rule).
 * `workspace` (device, 16-byte aligned, >= hpvm_sgemm_backward_workspace_bytes
 * for the same sizes, prec and tile) holds the partial sums of the scalars
 * and, for staged tiles, the bfloat16 planes.                              */
int hpvm_sgemm_backward_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t prec,
                                        const hpvm_tile* tile, int64_t* bytes);

int hpvm_sgemm_backward(int64_t m, int64_t n, int64_t k, float alpha, float beta, const float* A,
                        int64_t lda, const float* B, int64_t ldb, const float* C_in, int64_t ldci,
                        const float* G, int64_t ldg, float* dA, int64_t ldda, float* dB,
                        int64_t lddb, float* dC_in, int64_t lddci, float* dalpha, float* dbeta,
                        int32_t prec, const hpvm_tile* tile, void* workspace,
                        int64_t workspace_bytes, void* stream);

/* Tiles the backward can use at `prec` (writes at most `capacity`, total
 * count to *count).                                                         */
int hpvm_sgemm_backward_menu(int32_t prec, hpvm_tile* out, int32_t capacity, int32_t* count);

/* Autotuner of the backward: times dA + dB + dalpha (alpha = 1) for every
 * backward tile whose workspace fits (the last 256 bytes of `workspace` are
 * kept for a scratch dalpha), two rounds, `reps` calls each after a warm-up;
 * dA (m x k, ldda) and dB (k x n, lddb) are scratch outputs.  Records the
 * fastest for (prec, m, n, k), used when hpvm_sgemm_backward gets no tile.  */
int hpvm_autotune_backward(int64_t m, int64_t n, int64_t k, int32_t prec, const float* A,
                           int64_t lda, const float* B, int64_t ldb, const float* G, int64_t ldg,
                           float* dA, int64_t ldda, float* dB, int64_t lddb, void* workspace,
                           int64_t workspace_bytes, int32_t reps, void* stream, hpvm_tile* best,
                           float* best_ms);

/* ======================================================================== */
/* Autotuner of single launches                                             */
/* ======================================================================== */
/* The paper leaves tile sizes to the programmer and expects them to come
 * from "upstream optimization passes or autotuning tools" (Sec. 3.4).  This
 * tuner times every compiled tile of hpvm_tile_menu(prec) for one problem
 * with HIP events and records the fastest in a process-wide cache keyed by
 * (prec, m, n, k); the same entry also serves as the fallback for the shape
 * class (prec, ceil(log2 m), ceil(log2 n), ceil(log2 k)).  hpvm_sgemm with
 * tile == NULL takes the exact entry, else the class entry, else menu
 * entry 0.                                                                  */

/* Times the menu on A, B (device, read only) writing C_scratch (device,
 * m x n, leading dimension ldc; overwritten with beta = 0, never read).
 * Tiles of the staged lowering (stages == 3) are timed only when
 * `workspace` (device, 16-byte aligned) holds at least
 * hpvm_sgemm_workspace_bytes for them; DMA-fed tiles that split the
 * contraction run split when it holds their partial sums, and are then
 * left out of the no-workspace choice.  workspace may be NULL with 0 bytes.
 * Two rounds over the menu; in each, a tile runs once to warm up, then
 * `reps` times, and it keeps its faster round.  The cache records the
 * fastest tile (used by hpvm_sgemm_ws with tile == NULL) and the fastest
 * tile needing no workspace (used by hpvm_sgemm with tile == NULL).  Writes
 * the overall winner to *best (may be NULL) and its time per launch to
 * *best_ms (may be NULL).                                                   */
int hpvm_autotune(int64_t m, int64_t n, int64_t k, int32_t prec, const float* A, int64_t lda,
                  const float* B, int64_t ldb, float* C_scratch, int64_t ldc, void* workspace,
                  int64_t workspace_bytes, int32_t reps, void* stream, hpvm_tile* best,
                  float* best_ms);

/* Cache lookup of the overall winner: *found = 2 for an exact entry, 1 for
 * a shape-class entry, 0 when none is cached (then *tile is menu entry 0). */
int hpvm_autotune_lookup(int64_t m, int64_t n, int64_t k, int32_t prec, hpvm_tile* tile,
                         int32_t* found);

/* Records a choice without timing (e.g. from another process).  When the
 * tile needs a workspace, the no-workspace choice becomes menu entry 0.     */
int hpvm_autotune_record(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile,
                         float ms);

/* Empties the cache. */
int hpvm_autotune_clear(void);

/* Writes / merges the cache as text, one entry per line: the GPU
 * architecture and HIP runtime version it was timed with ("gfx950
 * hip<version>"), "prec m n k", the overall winner (tile_m tile_n tile_k
 * leaf_m leaf_n stages ms), then the no-workspace winner in the same form.
 * Loading skips entries timed on another architecture or runtime and
 * entries whose tiles are not compiled into this library.  With the
 * environment variable HPVM_AUTOTUNE_CACHE set to a path, the cache
 * persists there across processes: the file is merged in at the first use
 * of the cache (a missing file is an empty cache) and rewritten after every
 * hpvm_autotune and hpvm_autotune_record (processes sharing the file: the
 * last writer's entries win).  A save writes "<path>.tmp<pid>" and renames
 * it over the path, so a reader never sees a half-written file; a failed
 * save leaves the old file in place.                                       */
int hpvm_autotune_save(const char* path);
int hpvm_autotune_load(const char* path);

/* ======================================================================== */
/* Grouped launch: many independent sgemms in one persistent kernel         */
/* ======================================================================== */
/* The instances of a batch are independent dataflow graphs (Sec. 2.1: the
 * dynamic instances of a node are independent), so their SgemmInternal
 * tiles can share one launch.  One persistent kernel (Sec. 3.5 keeps nodes
 * alive as persistent workers; Sec. 4.2 fuses nodes to save kernel launches)
 * pulls tiles from a device-side list, longest first, with an atomic
 * counter; each instance has its own tile shape.  Plans are host objects;
 * device state lives in a caller-provided workspace.                       */

typedef struct hpvm_sgemm_desc {
  int64_t m, n, k;
  float alpha, beta;
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  float* C;
  int64_t ldc;
} hpvm_sgemm_desc;

typedef struct hpvm_grouped_info {
  int32_t count;        /* instances                                        */
  int32_t total_tiles;  /* SgemmInternal instances over the whole batch    */
  int32_t grid;         /* persistent workgroups per launch                */
  int32_t shapes_used;  /* distinct tile shapes in the plan                 */
  int64_t workspace_bytes;
  int64_t scratch_bytes; /* output scratch hpvm_grouped_autotune needs      */
  double flops;         /* sum of 2 m n k over the instances               */
} hpvm_grouped_info;

/* Validates every descriptor (the hpvm_sgemm rules per instance, and no two
 * instances' C ranges may overlap) and builds a plan.  prec must be
 * HPVM_PREC_FP32.  tile == NULL picks a shape per instance from
 * hpvm_grouped_menu with the built-in cost model; otherwise `tile` (from
 * that menu) is used for every instance.  Tuning the shapes is the separate
 * call hpvm_grouped_autotune rather than a flag here, so that creating a
 * plan never launches device work.  *plan receives an opaque handle
 * owned by the library until hpvm_grouped_plan_destroy.  The descriptors
 * are copied: the caller's array may be freed afterwards; the matrices
 * themselves must stay valid while the plan is run.                       */
int hpvm_grouped_plan_create(int32_t count, const hpvm_sgemm_desc* descs, int32_t prec,
                             const hpvm_tile* tile, void** plan);

/* Plan summary. */
int hpvm_grouped_plan_info(const void* plan, hpvm_grouped_info* info);

/* Tile shape chosen for instance `index` (0-based, in the caller's order). */
int hpvm_grouped_instance_tile(const void* plan, int32_t index, hpvm_tile* tile);

/* Shapes the grouped kernel supports (all 256 lanes per workgroup). */
int hpvm_grouped_menu(hpvm_tile* out, int32_t capacity, int32_t* count);

/* Device bytes the workspace of hpvm_grouped_run / _capture must have:
 * a tile counter, the instance descriptors and the tile -> instance map. */
int hpvm_grouped_workspace_bytes(const void* plan, int64_t* bytes);

/* Uploads the plan into `workspace` (device memory, >= the bytes above,
 * 16-byte aligned) and enqueues the batch on `stream`: a kernel that clears
 * the tile counter, then the persistent kernel.  Returns once enqueued.
 * Runs on one stream must not overlap in time on the same workspace.      */
int hpvm_grouped_run(void* plan, void* workspace, int64_t workspace_bytes, void* stream);

/* Uploads the plan into `workspace` (synchronously on `stream`) and builds
 * an instantiated HIP graph of the same two kernels (a counter-clearing
 * kernel, no memset node).  *graph receives a handle for hpvm_graph_launch;
 * the workspace and every matrix must stay valid while the graph exists.  */
int hpvm_grouped_capture(void* plan, void* workspace, int64_t workspace_bytes, void* stream,
                         void** graph);

/* Replays a graph on `stream` (asynchronous, like llvm.hpvm.launch; the
 * graph handle plays the role of the paper's graph ID, Table 1).           */
int hpvm_graph_launch(void* graph, void* stream);

/* Destroys a graph / plan.  Using a handle afterwards returns
 * HPVM_BAD_HANDLE.                                                          */
int hpvm_graph_destroy(void* graph);
int hpvm_grouped_plan_destroy(void* plan);

/* Autotuner of the grouped plan: times candidate shape assignments (one
 * shape for all instances, and the cost model's assignments over a range of
 * weights of the shapes' relative costs and of a fixed per-tile overhead,
 * each distinct assignment once) with the real kernel, keeps the fastest in
 * the plan and returns its time per launch in
 * *best_ms.  Timing runs use `scratch` (device memory of
 * hpvm_grouped_info.scratch_bytes, zeroed first) as every instance's C, with
 * the instance's own beta, so they read C where the replays do; the
 * instances' C are never touched.  Each candidate is launched `reps` times
 * after one warm-up.                                                       */
int hpvm_grouped_autotune(void* plan, void* workspace, int64_t workspace_bytes, float* scratch,
                          int64_t scratch_bytes, int32_t reps, void* stream, float* best_ms);

/* ======================================================================== */
/* Node fusion (Sec. 4.1 merge primitives, applied as in Sec. 4.2)           */
/* ======================================================================== */
/* Sec. 4.1 defines MergeDependentNodes (two leaves joined only by 1-1
 * edges become one leaf; the edges become assignments) and
 * MergeIndependentNodes (two leaves with the same parent and dimensions and
 * no path between them become one leaf); Sec. 4.2 uses them to fuse
 * kernels, for fewer launches and better reuse of data.  Two merges of the
 * sgemm leaf are offered here (FP32); independent sgemms that share no
 * operand merge into one launch with the grouped entry points above.      */

typedef enum hpvm_fusion {
  HPVM_FUSION_CONSUMER = 0,  /* sgemm leaf + 1-1 consumer leaf             */
  HPVM_FUSION_PAIR = 1       /* two sgemm leaves sharing input A           */
} hpvm_fusion;

/* The consumer leaf's function, applied to v = alpha (A B)_ij + beta C_ij:
 *   NONE       d = v
 *   RELU       d = v if v > 0, else 0   (NaN gives 0)
 *   BIAS       d = v + bias[j]
 *   BIAS_RELU  d = relu(v + bias[j])
 *   CLAMP      d = lo if v < lo, hi if v > hi, else v   (NaN stays NaN)  */
typedef enum hpvm_consumer_op {
  HPVM_CONSUMER_NONE = 0,
  HPVM_CONSUMER_RELU = 1,
  HPVM_CONSUMER_BIAS = 2,
  HPVM_CONSUMER_BIAS_RELU = 3,
  HPVM_CONSUMER_CLAMP = 4
} hpvm_consumer_op;

typedef struct hpvm_consumer {
  int32_t op;         /* hpvm_consumer_op                                   */
  int32_t reserved;   /* 0                                                  */
  const float* bias;  /* device, n floats (BIAS ops; else unused)          */
  float lo, hi;       /* CLAMP bounds, lo <= hi                             */
} hpvm_consumer;

/* Tiles compiled for a fusion: `which` is an hpvm_fusion.  For the pair,
 * tile_m x tile_n is the tile of each output.  Same conventions as
 * hpvm_tile_menu.                                                           */
int hpvm_fusion_menu(int32_t which, hpvm_tile* out, int32_t capacity, int32_t* count);

/* MergeDependentNodes(sgemm leaf, consumer leaf):
 *   D <- consumer(alpha * A B + beta * C)   element-wise, FP32,
 * in one launch; the sgemm result stays in registers.  A, B, C as in
 * hpvm_sgemm, except that C is only read (beta == 0: never read, may be
 * NULL).  D (m x n, leading dimension ldd >= max(1, n), device) receives
 * the consumer's output; it may be C itself (same pointer and leading
 * dimension) but may not otherwise overlap C, nor A, B or the bias vector.
 * tile: NULL = the autotuner's FP32 choice for the shape if it is in the
 * consumer menu, else hpvm_sgemm's built-in FP32 choice.  Errors as hpvm_sgemm, with
 * argument 12 the consumer (unknown op, NULL bias, lo > hi), 13/14 D.     */
int hpvm_sgemm_consumer(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda,
                        const float* B, int64_t ldb, float beta, const float* C, int64_t ldc,
                        const hpvm_consumer* consumer, float* D, int64_t ldd, const hpvm_tile* tile,
                        void* stream);

/* MergeIndependentNodes of two sgemm leaves whose parents share input A:
 *   C1 <- alpha1 A B1 + beta1 C1   and   C2 <- alpha2 A B2 + beta2 C2
 * (same m, n, k) in one launch; every workgroup stages one A tile and
 * computes the same tile of C1 and C2 from it.  Each output follows the
 * hpvm_sgemm rules (its checks run in that order, the detail text names
 * the output and the hpvm_sgemm argument position); C1 and C2 may not
 * overlap each other or the other output's B.  An output with k == 0 or
 * alpha == 0 shares nothing; the two outputs then take single launches.
 * tile: NULL = the first of the pair menu's 128 x 256 (DMA-fed),
 * 128 x 128 and 64 x 64 tiles per output that gives at least 256 tiles,
 * else 64 x 64.                                                             */
int hpvm_sgemm_pair(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, float alpha1,
                    const float* B1, int64_t ldb1, float beta1, float* C1, int64_t ldc1, float alpha2,
                    const float* B2, int64_t ldb2, float beta2, float* C2, int64_t ldc2,
                    const hpvm_tile* tile, void* stream);

/* hpvm_sgemm_pair with a workspace: pairs whose per-output tiles of the
 * first pair tile would not cover 256 CUs run on the DMA-fed 128 x 128
 * pair tile with the contraction split into slices (the rule of
 * hpvm_sgemm_ws: slices doubled while tiles * slices < 256, each a whole
 * number of 32-deep slabs and at least 256 deep, at most 16), each
 * workgroup computing one tile of both outputs over one slice from one A
 * slab; the raw partial sums go to `workspace` ([slice][m][n] of output 1,
 * then of output 2), then each output is formed as alpha * (sum of its
 * slices, in order) + beta * C.  Requires whole tiles (m, n multiples of
 * 128, k of 32 * slices), 16-byte aligned A, B1, B2, C1, C2 and leading
 * dimensions that are multiples of 4; otherwise, or with NULL or fewer
 * workspace bytes than hpvm_sgemm_pair_workspace_bytes gives, it runs as
 * hpvm_sgemm_pair.  workspace: device memory, 16-byte aligned, contents
 * are scratch.  tile: NULL = the choice above, else a pair menu tile
 * (split when it is the splitting tile and the workspace holds the
 * partial sums).  Every other argument and rule is hpvm_sgemm_pair's;
 * workspace is argument 19, workspace_bytes (>= 0) argument 20.            */
int hpvm_sgemm_pair_ws(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, float alpha1,
                       const float* B1, int64_t ldb1, float beta1, float* C1, int64_t ldc1,
                       float alpha2, const float* B2, int64_t ldb2, float beta2, float* C2,
                       int64_t ldc2, const hpvm_tile* tile, void* workspace,
                       int64_t workspace_bytes, void* stream);

/* Workspace bytes hpvm_sgemm_pair_ws needs for these sizes and tile (NULL =
 * the tile it would pick given enough): 2 * slices * m * n * 4 when it
 * splits the contraction, else 0.                                           */
int hpvm_sgemm_pair_workspace_bytes(int64_t m, int64_t n, int64_t k, const hpvm_tile* tile,
                                    int64_t* bytes);

/* ======================================================================== */
/* Streaming graph (llvm.hpvm.launch with Stream = 1, push, pop)              */
/* ======================================================================== */
/* Table 1 and Sec. 2.3 define the host intrinsics of a streaming graph:
 * launch with Stream = 1 returns a handle, push hands the graph one more
 * packed argument struct, pop returns the next output, in push order.
 * Sec. 3.5 makes the nodes of such a graph persistent: they stay alive and
 * process every item until the stream ends.  Here the graph is the sgemm
 * graph, its argument pack is an hpvm_sgemm_desc (FP32), and the persistent
 * node is one resident kernel on a stream of the library's own, reading the
 * pushed packs from pinned host memory.  Items in flight run concurrently
 * (the tiles of item i are handed out before those of item i + 1, but
 * nothing waits for item i to finish), so they must be independent.
 * While a stream is open its kernel is resident: a device-wide wait
 * (hipDeviceSynchronize, and calls that imply it such as hipFree) waits for
 * that kernel too, i.e. until the stream is closed or reaches its idle
 * limit.  Wait on streams or events instead.                                */

typedef struct hpvm_stream_config {
  int32_t capacity;  /* ring slots = most items pushed and not yet popped,
                        1..4096                                           */
  int32_t grid;      /* resident workgroups, 0..2 per compute unit of
                        the device (at most 512); 0 = two per compute
                        unit.  More is refused with HPVM_INVALID_ARG: a
                        third per compute unit would hold every SIMD's
                        registers, so no other kernel (a copy's included)
                        could start while the stream is open            */
  int32_t idle_ms;   /* the kernel ends the stream when nothing has been
                        pushed for this long, 1..60000                    */
  int32_t reserved;  /* 0                                                 */
} hpvm_stream_config;

typedef struct hpvm_stream_status {
  int64_t pushed, popped;
  int64_t tiles;       /* workgroup tiles of every item pushed so far      */
  int32_t capacity, grid, idle_ms;
  int32_t running;     /* 1 while the kernel has not exited                */
  int32_t idle_ended;  /* 1 if the kernel ended the stream at its idle
                          limit                                            */
  int32_t reserved;
} hpvm_stream_status;

/* Launches the persistent kernel on a new non-blocking stream of the
 * current device and returns its handle (the paper's graph ID).  The
 * library owns the handle, a small pinned host ring of `capacity` argument
 * slots, and 256 + 4 * capacity bytes of device memory, until
 * hpvm_stream_close.  At process exit every stream still open is closed
 * (bounded by its idle limit).  Errors: HPVM_INVALID_ARG for a field out of
 * range or NULL arguments; HPVM_HIP_ERROR if an allocation or the launch
 * fails (nothing is left running then).                                    */
int hpvm_stream_open(const hpvm_stream_config* config, void** handle);

/* Pushes one sgemm (llvm.hpvm.push).  The item is checked by the
 * hpvm_sgemm rules (sizes, leading dimensions, NULLs, C overlapping its own
 * A or B) and must not overlap an item in flight: its C may not meet
 * another in-flight item's A, B or C, and its A and B may not meet another
 * in-flight item's C (HPVM_INVALID_ARG).  The matrices must stay valid
 * until the item is popped.  HPVM_QUEUE_FULL when `capacity` items are in
 * flight (pop first); HPVM_STREAM_ENDED once the kernel has exited.
 * *seq (may be NULL) receives the item's sequence number, 0, 1, 2, ...    */
int hpvm_stream_push(void* handle, const hpvm_sgemm_desc* item, int64_t* seq);

/* Pops the oldest item in flight once it is complete (llvm.hpvm.pop):
 * *seq receives its sequence number and *C its output pointer (either may
 * be NULL).  Its C is then final and visible to later work on any stream.
 * Waits at most timeout_ms (0 = just test): HPVM_TIMEOUT leaves the item in
 * flight.  HPVM_INVALID_ARG if nothing is in flight; HPVM_STREAM_ENDED if
 * the kernel exited before the item completed (its idle limit, or a ticket
 * map entry naming a slot past the ring, which the library never writes:
 * the kernel then ends the stream instead of reading past the ring);
 * HPVM_HIP_ERROR if it failed.                                              */
int hpvm_stream_pop(void* handle, int32_t timeout_ms, int64_t* seq, float** C);

/* Counters and state of a stream.                                          */
int hpvm_stream_info(const void* handle, hpvm_stream_status* info);

/* Ends the stream: the kernel finishes every item already pushed, then
 * exits; the call waits for that at most timeout_ms and then frees the
 * stream's resources and the handle (later use: HPVM_BAD_HANDLE).
 * HPVM_TIMEOUT if the kernel is still draining (the handle stays valid;
 * close again).  Unpopped items are dropped after they complete.          */
int hpvm_stream_close(void* handle, int32_t timeout_ms);

/* ======================================================================== */
/* Memory tracker for host-resident arrays                                   */
/* ======================================================================== */
/* Sec. 2.3 ("Performance features") has the runtime record where the latest
 * copy of each data array lives, so that copies between address spaces
 * happen only when needed; node arguments marked in / out / inout tell it
 * which copies a launch needs, and host code uses track / request / untrack
 * explicitly (the runtime calls listed there and used by the host code of
 * the Sec. 6.1 listing).  Here the tracked regions are host memory (pinned
 * or pageable) and the library keeps one device copy per region, allocated
 * on first use, stream-ordered, on the stream of that call.  The table is
 * process-wide and guarded by a lock; a region must not be untracked while
 * a launch that uses it is being enqueued on another thread.             */

typedef struct hpvm_tracked {
  void* start;        /* host start of the region holding the pointer    */
  int64_t bytes;
  void* device;       /* its device copy, NULL before first use           */
  int32_t on_host;    /* 1 when the host copy is current                  */
  int32_t on_device;  /* 1 when the device copy is current                */
} hpvm_tracked;

typedef struct hpvm_tracker_stats {
  int64_t h2d_bytes, h2d_copies;  /* copies made so far, process-wide    */
  int64_t d2h_bytes, d2h_copies;
  int64_t launches;               /* hpvm_sgemm_tracked launches          */
  int64_t regions;                /* regions tracked now                  */
} hpvm_tracker_stats;

/* llvm_hpvm_track_mem: adds [ptr, ptr + bytes) of host memory to the table,
 * with the host copy current.  HPVM_INVALID_ARG for NULL, bytes <= 0, or a
 * region overlapping one already tracked.                                 */
int hpvm_track_mem(void* ptr, int64_t bytes);

/* llvm_hpvm_request_mem: the host is about to access [ptr, ptr + bytes).
 * If the latest copy of the region holding it is on the device, the whole
 * region is copied back on `stream` and the call waits for it; otherwise
 * nothing happens.  HPVM_INVALID_ARG if the range is not inside one tracked
 * region.                                                                  */
int hpvm_request_mem(void* ptr, int64_t bytes, void* stream);

/* llvm_hpvm_untrack_mem: removes the region starting at ptr; its device
 * copy is freed stream-ordered on `stream`, after the work queued there and
 * on the stream that allocated it.  The host copy is left as it is (request
 * it first to keep the device's latest data).                             */
int hpvm_untrack_mem(void* ptr, void* stream);

/* Where the latest copy of the region holding ptr lives.                  */
int hpvm_tracked_state(const void* ptr, hpvm_tracked* out);
int hpvm_tracker_counters(hpvm_tracker_stats* out);

/* The sgemm root launch on host arrays, as the host code of the Sec. 6.1
 * listing runs it: A, B and C are host pointers inside tracked regions.
 * A and B are `in` (copied to the device only when their device copy is
 * stale), C is `in out` (copied in unless the node overwrites its whole
 * region: beta == 0, ldc == n and the region is exactly C); after the
 * launch the latest C is on the device, until hpvm_request_mem.  Checks as
 * hpvm_sgemm, then HPVM_INVALID_ARG for an untracked operand (argument 5,
 * 7 or 10).  The copies and the launch are enqueued on `stream`.          */
int hpvm_sgemm_tracked(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda,
                       const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int32_t prec,
                       const hpvm_tile* tile, void* stream);

/* ======================================================================== */
/* CPU (vector) lowering of the same graph                                   */
/* ======================================================================== */
/* The paper compiles one graph to GPUs, to the vector units of a CPU and to
 * host threads (Sec. 3.3, evaluated in Sec. 5).  This is the sgemm graph
 * lowered by hand onto host cores: SgemmInternal instances are tile_m x
 * tile_n tiles of C pulled by worker threads, the Allocation node is each
 * worker's packed tile_k panels of A and B, and SgemmLeaf instances are a
 * leaf_m x leaf_n block of outputs in vector registers.  FP32 arithmetic.
 * A separate target: no GPU entry point ever calls it.                    */

/* The compiled CPU tiles (stages = 1); entry 0 is the default.            */
int hpvm_cpu_menu(hpvm_tile* out, int32_t capacity, int32_t* count);

/* The instruction set the micro-kernel runs with on this host ("avx512f",
 * "avx2" or "x86-64").                                                      */
const char* hpvm_cpu_isa(void);

/* C <- alpha A B + beta C on host memory, synchronously, with `threads`
 * workers (0 = the host's cores, capped by OMP_NUM_THREADS when set).
 * Arguments and errors as hpvm_sgemm (host pointers); tile NULL = the
 * default, else one of hpvm_cpu_menu (HPVM_UNSUPPORTED otherwise).        */
int hpvm_sgemm_cpu(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda,
                   const float* B, int64_t ldb, float beta, float* C, int64_t ldc, const hpvm_tile* tile,
                   int32_t threads);

/* ======================================================================== */
/* Diagnostics                                                               */
/* ======================================================================== */

/* Static text for a status code. */
const char* hpvm_status_string(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char* hpvm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HPVM_SGEMM_H */
