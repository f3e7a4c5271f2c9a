/*
 * gee.h — C ABI of the MI355X (gfx950) one-hot graph encoder embedding library.
 *
 * The operation is Algorithm 1 ("Semi-Supervised GEE") of Lubonja, Shen, Priebe
 * and Burns, "Edge-Parallel Graph Encoder Embedding", Section II: given an edge
 * list E of s records (u, v, w) and labels Y in {0..K}^n (0 = unknown class),
 * build the projection W(v, k) = 1 / count(Y = k) for Y(v) = k, then in one pass
 * over the records add W(v, Y(v)) * w to Z(u, Y(v)) and W(u, Y(u)) * w to
 * Z(v, Y(u)). Section II calls this the formulation for weighted directed graphs;
 * unweighted graphs use w = 1. The result is Z = (A + A^T) M with A[u][v] the sum
 * of w over records (u, v) and M[v][k-1] = [Y(v) = k] / n_k.
 *
 * The Laplacian version, whose preprocessing Section II leaves out, scales each
 * record's w by (d_u d_v)^-1/2 with d = (A + A^T) 1 the weighted degree:
 * Z = D^-1/2 (A + A^T) D^-1/2 M, and a vertex of degree 0 gets factor 0.
 *
 * Conventions shared by every entry point:
 *  - Vertex ids are 0-based int32 in [0, n), n <= 2^31 - 1.
 *  - Labels are int32 in [0, K], 1 <= K <= 65535; class k in 1..K is column
 *    k - 1 of Z; an update whose target class is 0 is skipped, the record's
 *    other update still happens. Self-loops fire both updates, repeated records
 *    add up.
 *  - Z is FP32, n x K, row-major: Z[u * K + (k - 1)].
 *  - Unless marked "host", every pointer is device memory on the current HIP
 *    device, owned by the caller. The library allocates no device memory: the
 *    calls that need scratch take a caller-provided workspace of the size the
 *    matching *_workspace() query returns, aligned to 256 bytes (gee_embed_noalloc
 *    instead uses a static array the library holds on each device).
 *  - Every call is stream-ordered on `stream` and returns before the GPU work
 *    finishes. Inputs must stay valid, and outputs untouched, until then.
 *  - Calls are stateless and reentrant; calls on different streams with
 *    disjoint outputs and workspaces are independent.
 *
 * Errors come in two classes:
 *  - host-detectable ones (bad sizes, null pointers, short workspace) are
 *    returned at once and nothing is launched;
 *  - data-dependent ones (a label outside [0, K], a vertex id outside [0, n),
 *    a negative weight in the Laplacian version) are found by the kernels that
 *    already read the data. The offending item is skipped and the lowest code
 *    seen is stored into the caller's device word `*err` by atomic minimum. The
 *    library never resets `*err`: the caller zeroes it before the call and reads
 *    it after synchronising. When `*err != 0` the outputs are unspecified.
 */
#ifndef GEE_H
#define GEE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GEE_OK = 0,
    GEE_EINVAL = -1,     /* bad argument: null pointer, size out of range, bad option */
    GEE_ELABEL = -2,     /* a label outside [0, K] (data-dependent) */
    GEE_EVERTEX = -3,    /* a vertex id outside [0, n) (data-dependent) */
    GEE_ENEGW = -4,      /* a negative or NaN weight in the Laplacian version (data-dependent) */
    GEE_EOVERFLOW = -5,  /* n * K or an index would overflow 64 bits / the supported range */
    GEE_EWORKSPACE = -6, /* workspace null, misaligned or smaller than the query says */
    GEE_EHIP = -7        /* a HIP launch or event call failed */
} gee_status;

/* Edge list of s records (src[i], dst[i], w[i]), i < s. w == NULL means unit
 * weights. The struct itself is host memory; the arrays are device memory. */
typedef struct gee_coo {
    int64_t n;          /* vertex count, 1 <= n <= 2^31 - 1 */
    int64_t s;          /* record count, s >= 0 */
    const int32_t *src; /* [s] */
    const int32_t *dst; /* [s] */
    const float *w;     /* [s] or NULL */
} gee_coo;

/* Symmetric CSR of S = A + A^T (the per-vertex edge lists that the paper's
 * edge-map walks, Section III): for record (u, v, w), row u holds (v, w) and row
 * v holds (u, w); a self-loop appears twice in its row. row_ptr is
 * non-decreasing with row_ptr[0] = 0 and row_ptr[n] = nnz. gee_csr_build writes
 * rows sorted by (column, bit pattern of w), which makes the layout independent
 * of record order; gee_embed accepts any valid layout. val == NULL means unit
 * weights. The struct is host memory; the arrays are device memory.
 *
 * Hot-vertex slots (optional, n_hot > 0): a column value with bit 31 set names
 * slot (col & 0x7fffffff) < n_hot, whose vertex is hot_ids[slot]. gee_csr_build
 * gives the n_hot highest-degree vertices such slots so that gee_embed gathers
 * their labels from a compact table that stays in cache. With n_hot == 0 every
 * column is a plain vertex id and hot_ids is ignored. */
typedef struct gee_csr {
    int64_t n;              /* vertex count, as in gee_coo */
    int64_t nnz;            /* entry count (2 s for a CSR built from s records) */
    const int64_t *row_ptr; /* [n + 1] */
    const int32_t *col;     /* [nnz] */
    const float *val;       /* [nnz] or NULL */
    int64_t n_hot;          /* number of hot slots, 0 <= n_hot <= n */
    const int32_t *hot_ids; /* [n_hot] vertex id of each slot, or NULL when n_hot == 0 */
} gee_csr;

/* Optional knobs of gee_embed (host struct; pass NULL for the defaults). */
typedef struct gee_embed_opts {
    /* CSR-pull form: work items (rows + entries) per wavefront segment; 0 picks
     * the default: the power of two at or above (n + nnz) / 131072 within
     * [1024, 16384], so that small graphs still give the GPU enough wavefronts
     * (it depends only on the graph). Must be 0 or in [64, 65535]. */
    int32_t seg_len;
    /* CSR-pull form: rows per LDS window; 0 picks the largest that fits the
     * per-wavefront LDS budget (at most 64). Must be 0 or in [1, 64]. */
    int32_t rows_per_window;
    /* When non-NULL, recorded on `stream` right before and right after the launch
     * of the edge-pass kernel (push or pull), so a caller can time that kernel
     * alone. */
    hipEvent_t hot_begin;
    hipEvent_t hot_end;
    /* Batched form: at most this many vectors per group (the label tile: fewer vectors
     * per group mean fewer FP64 bins per wavefront and more wavefronts per CU, but one
     * more pass over the CSR per group); 0 picks 64. Must be 0 or in [1, 64]. A
     * vector's result does not depend on its group. */
    int32_t group_vectors;
} gee_embed_opts;

/* Class counts, Algorithm 1's count(Y = k): counts[k] = #{v : labels[v] = k} for
 * k = 0..K (index 0 counts unknown labels). labels: [n] int32; counts: [K + 1]
 * int64, overwritten. A label outside [0, K] is not counted and raises
 * GEE_ELABEL in *err. */
int gee_counts(const int32_t *labels, int64_t n, int32_t K, int64_t *counts, int32_t *err,
               hipStream_t stream);

/* Projection weights, Algorithm 1's W(idx, k) = 1 / count(Y = k), stored as one
 * value per class: inv[0] = 0, inv[k] = 1 / counts[k] (IEEE-754 FP64 division,
 * correctly rounded) or 0 when counts[k] = 0. W itself is never materialised:
 * W(v, k) = [labels[v] = k] * inv[k]. counts: [K + 1] int64; inv: [K + 1] double. */
int gee_weights(const int64_t *counts, int32_t K, double *inv, hipStream_t stream);

/* Weighted degree d = (A + A^T) 1 (a self-loop adds 2 w), the preprocessing of
 * the Laplacian version. With csr != NULL the rows of the CSR are summed in FP64,
 * each in a fixed order (bit-reproducible): its stored order, except that a row of
 * more than 4,096 entries is summed as 64 interleaved partial sums that are then
 * added pairwise. Otherwise the records of g are accumulated with FP64 atomics.
 * Both are exact for unit weights, and for weights on a 2^-k grid whose sums stay
 * below 2^(53-k). deg: [n] double, overwritten. Exactly the graph given is read: g
 * may be NULL when csr is not, and vice versa. */
int gee_degrees(const gee_coo *g, const gee_csr *csr, double *deg, int32_t *err, hipStream_t stream);

/* Workspace bytes gee_embed needs for this graph, K and variant (csr == NULL:
 * edge-parallel push form; else CSR-pull form). Returns 0 on invalid input. */
size_t gee_embed_workspace(const gee_coo *g, const gee_csr *csr, int32_t K, int laplacian,
                           const gee_embed_opts *opts);

/* The embedding Z (Algorithm 1; Laplacian version when laplacian != 0).
 *  csr == NULL: edge-parallel push form. One thread per record gathers both
 *    endpoints' labels and adds into Z with FP32 global atomics; class weights
 *    and the row factor of the Laplacian are applied by a final scaling pass.
 *    Needs g. Unit-weight adjacency sums are exact integers before the one
 *    final rounding; other sums round in FP32 in an unspecified order.
 *  csr != NULL: CSR-pull form. Rows are split into segments of equal work
 *    (rows + entries); one wavefront per segment accumulates each row's K bins in
 *    LDS and writes every row of Z exactly once; a row cut by segment boundaries
 *    is summed from FP64 partials in segment order by a second pass. Bit-identical
 *    from run to run. Needs csr (g unused, may be NULL); K <= 4096.
 * Z: [n * K] float, overwritten (no zero-fill needed). ws: workspace of at least
 * gee_embed_workspace() bytes. */
int gee_embed(const gee_coo *g, const gee_csr *csr, const int32_t *labels, int32_t K, int laplacian,
              float *Z, void *ws, size_t ws_bytes, int32_t *err, const gee_embed_opts *opts,
              hipStream_t stream);

/* Bytes of the scratch that gee_embed_noalloc uses: one static device array of this
 * size on every GPU the library runs on, held until the process ends. */
#define GEE_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (work recorded into a HIP graph,
 * tight serving loops, harnesses that forbid hipMalloc): gee_embed with the library's
 * own static scratch in place of the workspace argument. Same arguments (minus ws and
 * ws_bytes), forms, results and errors as gee_embed; the kernels are the same. Calls
 * no hipMalloc, hipFree or other allocating routine. GEE_EWORKSPACE, with nothing
 * launched, when gee_embed_workspace() for these arguments exceeds
 * GEE_NOALLOC_SCRATCH_BYTES. The first call on a device looks up that device's scratch
 * address (GEE_EHIP if that fails). Every call on one GPU shares that GPU's scratch,
 * which keeps the last call's contents (the call clears what it needs zeroed itself):
 * calls that overlap in time on one GPU, on any streams, race and give wrong results;
 * order them on one stream or synchronise between them. */
int gee_embed_noalloc(const gee_coo *g, const gee_csr *csr, const int32_t *labels, int32_t K, int laplacian,
                      float *Z, int32_t *err, const gee_embed_opts *opts, hipStream_t stream);

/* ------------------------------------------------------------------------------
 * Propagation-blocked layout of a CSR, and the pull pass over it.
 *
 * The pull pass of Algorithm 1 (Section II; Section III's per-vertex edge lists)
 * reads the label of every entry's column at a random address. The adjacency
 * version only needs, per entry, its row, its weight and the label of its column,
 * so the entries can be re-laid out once per graph: sorted stably by column block
 * (2^21 vertices), each entry keeping its column, its row within a block of 256 rows
 * and, for a weighted CSR, its weight.
 * Entries whose column is one of the CSR's first n_lds hot slots (its highest-degree
 * vertices, n_lds <= 2^26) go instead to "tier slices" of 2^17 slots each, one extra
 * column block per slice after the vertex blocks, and keep their slot within the
 * slice. Per call, one streaming pass writes every entry's label in that order (a
 * vertex block's labels stay in L2; a slice's labels, 128 KB, are read from LDS) and
 * a second pass counts, per 256-row block, the (row, class) pairs of the block's
 * cells in LDS and writes those rows of Z once. Unit-weight counts are integers: Z
 * is bit-identical to gee_embed on the same CSR. With weights the second pass adds
 * them into FP64 sums. When every positive weight is an integer multiple of one power of
 * two 2^-g and a sum of 128 of them, scaled by 2^g, stays below 2^32 (the build records g
 * in meta[4]), the row blocks whose rows have at most 128 entries and no negative weight
 * (rb_flag 0) add the scaled weights in 32-bit integers instead, which is exact (weights
 * on the 2^-24 grid in (0, 1] qualify). Otherwise results agree with gee_embed within
 * rounding, not bit for bit, and since a block's wavefronts add into shared bins in an
 * order that varies, two calls agree within rounding too (the CSR pull form of gee_embed
 * is the bit-reproducible one).
 *
 * A Laplacian layout (gee_pb_build with laplacian != 0) stores, in place of the weights,
 * each entry's w d_u^-1/2 d_v^-1/2 (both its row's and its column's factor, FP32: the
 * product of the FP32 weight and the two FP32 factors rounded once) and every vertex's
 * d^-1/2 (rsd), the degrees d = (A + A^T) 1 being taken once when the layout is built, as
 * the CSR is (they depend on the graph only). The pass then adds the stored terms as a
 * weighted layout does: the Laplacian version, within the same rounding bound.
 *
 * Cell (rb, cb) of the layout is the run of column block cb's entries whose rows
 * lie in [256 rb, 256 rb + 256); cell_start[rb * n_cb + cb] is its first index in
 * the layout and cell_count[...] its length. The tier's entries start at H0, the
 * first multiple of 16 at or after the end of the vertex blocks (the gap before it
 * belongs to no cell); with NT tier entries padded to NTp, a multiple of 64, tier entry
 * i keeps the low 16 bits of its slot in bytes 4 H0 + 2 (i - H0) .. + 1 of col
 * (little-endian) and its 17th bit as bit (i - H0) mod 8 of byte 4 H0 + 2 NTp +
 * (i - H0) / 8 (8-byte aligned). n_rb = ceil(n / 256),
 * n_cb = ceil(n / 2^21) + ceil(n_lds / 2^17). The layout holds at most 2^32 - 65
 * entries (GEE_EOVERFLOW beyond).
 * ------------------------------------------------------------------------------ */
#define GEE_PB_SLICE 131072        /* hot slots per tier slice */
#define GEE_PB_MAX_TIER 67108864   /* at most 512 slices */

typedef struct gee_pb {
    int64_t n, nnz;            /* vertices, entries (as in the CSR) */
    int64_t n_rb;              /* row blocks */
    int32_t n_cb;              /* column blocks: vertex blocks, then tier slices */
    const int32_t *col;        /* [nnz + 64] layout order, 16-byte aligned: the column of each vertex-block entry;
                                  each tier entry's slot within its slice (17 bits) from byte 4 H0 on */
    const uint8_t *ul;         /* [nnz + 32 rounded up to 16] row within its 256-row block; 16-byte aligned */
    const int64_t *cell_start; /* [n_rb * n_cb] */
    const uint32_t *cell_count; /* [n_rb * n_cb] */
    int64_t n_lds;             /* tier slots the layout was built with (0 to GEE_PB_MAX_TIER) */
    const int32_t *lds_ids;    /* [n_lds] vertex of each tier slot (written by gee_pb_build) */
    const uint32_t *cell_word; /* [n_rb * n_cb] first 32-bit word of each cell within its row block's words */
    const float *val;          /* [nnz + 32 rounded up to 16] layout order, 16-byte aligned: the weight of each
                                  entry; NULL for a unit-weight layout */
    const uint8_t *rb_flag;    /* [n_rb] weighted layouts: 1 where a row of the block has more than 128 entries
                                  or a negative weight (FP64 sums), else 0; NULL for a unit-weight layout */
    const int64_t *meta;       /* [8] written by gee_pb_build: n, nnz, n_lds, the kind (0 unit-weight
                                  adjacency, 1 weighted adjacency, 2 Laplacian), then the weights' grid
                                  (below). A layout whose meta disagrees with the fields here (one built
                                  for another graph) makes gee_embed_pb skip its passes and raise
                                  GEE_EVERTEX */
    const float *rsd;          /* [n] Laplacian layouts: d^-1/2 of every vertex (0 where d = 0); else NULL */
} gee_pb;

/* n_rb * n_cb for n vertices and n_lds tier slots (0 on invalid input). */
int64_t gee_pb_cells(int64_t n, int64_t n_lds);

/* A tier size for the layout of csr: the hot slots of the longest run of leading
 * slices (at most 512, of min(n_hot, GEE_PB_MAX_TIER) slots) whose entries average at
 * least min_per_row_block per 256-row block, since each slice adds one cell to every
 * row block. Counts each slice's entries on the GPU (row lengths of its vertices) in
 * ws (device, 256-byte aligned, at least 4096 bytes) and SYNCHRONIZES the stream.
 * Returns the slot count (0 for no tier) or a negative status. */
int64_t gee_pb_tier_slots(const gee_csr *csr, int64_t min_per_row_block, void *ws, size_t ws_bytes,
                          hipStream_t stream);

/* Scratch bytes gee_pb_build needs (0 on invalid input, more than 2^32 - 65 entries,
 * or n_lds above min(n_hot, GEE_PB_MAX_TIER)). */
size_t gee_pb_build_workspace(const gee_csr *csr, int64_t n_lds, int laplacian);

/* Builds the layout of csr with the first n_lds hot slots (0 <= n_lds <=
 * min(n_hot, GEE_PB_MAX_TIER)) in the tier, for the adjacency version (laplacian = 0)
 * or the Laplacian version; other hot-slot columns are decoded through hot_ids. Outputs
 * are caller device buffers: col [nnz + 64] (16-byte aligned), ul [nnz + 32 rounded up
 * to 16] (16-byte aligned), cell_start, cell_count and cell_word [gee_pb_cells(n,
 * n_lds)], lds_ids [n_lds] (may be NULL when n_lds = 0), meta [8]; for a weighted CSR
 * (csr->val != NULL) or a Laplacian layout also val [nnz + 32 rounded up to 16]
 * (16-byte aligned) and rb_flag [ceil(n / 256)], and for a Laplacian layout rsd [n];
 * each must be NULL when not needed. cell_word[rb * n_cb + c] is the first 32-bit word
 * of cell c when the cells of row block rb are read one after another as words (a cell
 * covering ceil(((cell_start mod 4) + cell_count) / 4) of them, none when empty). A
 * column id outside [0, n) stores GEE_EVERTEX in *err; for a Laplacian layout a
 * negative or NaN weight stores GEE_ENEGW. */
int gee_pb_build(const gee_csr *csr, int64_t n_lds, int laplacian, int32_t *col, uint8_t *ul, int64_t *cell_start,
                 uint32_t *cell_count, uint32_t *cell_word, int32_t *lds_ids, float *val, uint8_t *rb_flag,
                 float *rsd, int64_t *meta, void *ws, size_t ws_bytes, int32_t *err, hipStream_t stream);

/* Workspace bytes of gee_embed_pb (0 on invalid input); 1 <= K <= 255. */
size_t gee_embed_pb_workspace(const gee_pb *pb, int32_t K);

/* Algorithm 1 over the layout, in the version the layout was built for: labels [n] in
 * [0, K] (K <= 255), Z [n * K] FP32 overwritten. Same results and data errors as
 * gee_embed on the CSR the layout was built from (bit for bit for unit-weight
 * adjacency; otherwise within the rounding described above). opts->hot_begin / hot_end
 * bracket the two passes (label gathers and row sums); seg_len is unused. */
int gee_embed_pb(const gee_pb *pb, const int32_t *labels, int32_t K, float *Z, void *ws, size_t ws_bytes,
                 int32_t *err, const gee_embed_opts *opts, hipStream_t stream);

/* DIAGNOSTIC, NOT THE EMBEDDING: the push form of gee_embed (g required, csr not
 * used) with every update of Z a plain read-modify-write instead of an atomic add.
 * Concurrent updates of one element race and can be lost, so Z is wrong whenever
 * two records of the list update the same element (it is exact when none do, and
 * for non-negative contributions never above the true value). It reproduces the
 * paper's atomics-off run (Section IV: the program run with unsafe updates to
 * measure what the atomics cost) and exists only for that measurement. Arguments,
 * workspace (gee_embed_workspace with csr = NULL) and errors as for gee_embed. */
int gee_embed_push_nonatomic(const gee_coo *g, const int32_t *labels, int32_t K, int laplacian, float *Z, void *ws,
                             size_t ws_bytes, int32_t *err, const gee_embed_opts *opts, hipStream_t stream);

/* A batch of label vectors over one graph. Vector b has labels
 * labels[b * n .. b * n + n) in [0, K[b]], the Laplacian version when laplacian[b]
 * != 0, and its n x K[b] embedding block at Z[u * ldz + zoff[b] + (k - 1)]. The
 * column blocks of different vectors must not overlap. Host struct; labels and Z
 * are device memory, K, laplacian and zoff host arrays. */
typedef struct gee_batch {
    int32_t B;                /* number of vectors, 1 <= B <= 4096 */
    const int32_t *labels;    /* [B * n] int32 */
    const int32_t *K;         /* [B], 1 <= K[b] <= 4096 */
    const int32_t *laplacian; /* [B] */
    const int64_t *zoff;      /* [B] first column of each block, zoff[b] + K[b] <= ldz */
    int64_t ldz;              /* floats per row of Z */
    float *Z;                 /* [n * ldz] */
} gee_batch;

/* Workspace bytes gee_embed_batch needs for this graph and batch (0 on invalid input). */
size_t gee_embed_batch_workspace(const gee_csr *csr, const gee_batch *batch, const gee_embed_opts *opts);

/* Batched Algorithm 1: every vector of the batch embedded over one graph with one
 * pass of the CSR per group of vectors. Vectors taken in column order whose blocks
 * are contiguous form groups of up to opts->group_vectors (default 64) with at most
 * 4096 classes in total, any mix of adjacency and Laplacian vectors; the group's
 * labels are stored transposed, one row per vertex (8-bit labels when every vector of
 * the group has K <= 255, else 16-bit), so one gather of a neighbour's row serves the
 * whole group, and each row of Z gets the group's columns written once. Every bin is an FP64 sum
 * taken in CSR order, so results are bit-reproducible. Vector b's block holds the
 * values gee_embed returns for it (identical bits for unit-weight adjacency
 * vectors; other sums may differ in rounding order). Laplacian vectors share one
 * degree pass. Per-segment work follows opts->seg_len as in gee_embed, except that
 * 0 picks the power of two at or above (n + nnz) / 32768 within [512, 16384] (its
 * lanes are vectors, so a wavefront walks a segment's entries one at a time and
 * short segments keep the GPU busy; the choice depends only on the graph);
 * opts->hot_begin / hot_end bracket the group passes (label packing, edge pass and
 * split-row merge of every group). Data errors as for gee_embed; columns of Z
 * outside the blocks are not touched. GEE_EINVAL also when ldz > 2^31 - 1. */
int gee_embed_batch(const gee_csr *csr, const gee_batch *batch, void *ws, size_t ws_bytes, int32_t *err,
                    const gee_embed_opts *opts, hipStream_t stream);

/* Workspace bytes gee_csr_build needs (weighted != 0 when the records carry w;
 * hot_budget as passed to gee_csr_build). Returns 0 on invalid input. */
size_t gee_csr_workspace(int64_t n, int64_t s, int weighted, int64_t hot_budget);

/* Build the symmetric CSR of S = A + A^T from g: row_ptr [n + 1] int64, col [2 s]
 * int32 and, when g->w != NULL, val [2 s] float (else val may be NULL). Rows come
 * out sorted by (column, bit pattern of w): a stable LSD radix sort of the 2 s
 * directed entries, so the result depends only on the multiset of records.
 * With hot_budget > 0, the n_hot = min(hot_budget, n) vertices of highest degree
 * get slots 0..n_hot-1 in order of degree (capped at 4095), highest first, ties by
 * smaller id: hot_ids [n_hot] receives their ids and each column naming one of
 * them is stored as (slot | 0x80000000); the gee_csr passed to gee_embed then
 * carries n_hot and hot_ids. The choice of slots depends only on the graph. */
int gee_csr_build(const gee_coo *g, int64_t hot_budget, int64_t *row_ptr, int32_t *col, float *val,
                  int32_t *hot_ids, void *ws, size_t ws_bytes, int32_t *err, hipStream_t stream);

/* Labels from an embedding (Section II: labels may be known ground truth or the
 * output of a clustering; Section I: embeddings serve classification and clustering).
 * labels[u] = 1 + the first k with Z[u][k] equal to the largest entry of row u when
 * that entry is above zero, else 0 (no labelled neighbour): each vertex takes the
 * class to which it has the most weight per class member. Z is [n * ldz] (K <= ldz
 * columns used), labels [n] int32. When prev is given, *changed (a device word, may
 * be NULL) receives the number of vertices whose label differs from prev[u]; labels
 * and prev must not overlap. Launches kernels only, so it can be recorded. */
int gee_argmax(const float *Z, int64_t n, int32_t K, int64_t ldz, const int32_t *prev, int32_t *labels,
               uint64_t *changed, hipStream_t stream);

/* Segment length and label tile for gee_embed_batch on this graph and batch (the
 * autotuner of the batched form): for each pair of a candidate length in seg_lens
 * (host array of n_seg, each a multiple of 64, at most 2^22, or 0 for the library's
 * choice) and a candidate group size in group_vectors (host array of n_group, each 0
 * or in [1, 64]; NULL with n_group = 0 tries only the default 64) it makes one
 * untimed call, then reps timed calls bracketed by HIP events on stream, and returns
 * the fastest pair in *best_seg and *best_group and its mean time per call in
 * *best_ms (host pointers). ws must hold gee_embed_batch_workspace() for every pair.
 * The batch's Z receives the result of the last pair's calls (for unit-weight
 * adjacency vectors the same bits with any pair; other sums may differ in rounding
 * order with the segment length). SYNCHRONIZES the stream; returns a status code. */
int gee_embed_batch_tune(const gee_csr *csr, const gee_batch *batch, const int32_t *seg_lens, int n_seg,
                         const int32_t *group_vectors, int n_group, int reps, void *ws, size_t ws_bytes, int32_t *err,
                         hipStream_t stream, int32_t *best_seg, int32_t *best_group, float *best_ms);

/* ------------------------------------------------------------------------------
 * Recording repeated calls as a HIP graph. A sequence of calls that runs again and
 * again on the same buffers (the passes of a clustering loop over one graph, a
 * serving step of fixed shape) can be recorded once and replayed with one launch,
 * which removes the host cost of its many kernel launches. Between gee_capture_begin
 * and gee_capture_end on a stream (not the null stream) the gee_* calls made on that
 * stream by this host thread are recorded, not run; their arguments, pointers
 * included, are fixed at that point, and each replay reads whatever the buffers hold
 * then (new labels, say). The embedding and CSR entry points record cleanly (they
 * launch kernels only, with no memset or host synchronization); gee_pb_tier_slots
 * synchronizes and must not be recorded. The data-error word is not reset by a
 * replay: clear it between replays if it is read.
 * ------------------------------------------------------------------------------ */
typedef struct gee_graph gee_graph; /* opaque; host memory */

/* Starts recording on stream (GEE_EINVAL for the null stream). */
int gee_capture_begin(hipStream_t stream);

/* Ends recording on stream and instantiates what was recorded; *graph receives the
 * handle, or NULL on failure (a failed or unrecordable call inside; the recording is
 * then discarded). */
int gee_capture_end(hipStream_t stream, gee_graph **graph);

/* Enqueues one replay of graph on stream. */
int gee_graph_launch(const gee_graph *graph, hipStream_t stream);

/* Frees graph (NULL is ignored); no replay of it may still be pending. */
void gee_graph_destroy(gee_graph *graph);

/* Measurement probe: copy `bytes` bytes from src to dst with a plain streaming
 * kernel (16-byte loads and stores). Used to calibrate memory-traffic counters
 * and to measure the attainable copy bandwidth. Both pointers 16-byte aligned. */
int gee_copy(void *dst, const void *src, size_t bytes, hipStream_t stream);

/* Host: static description of a status code. */
const char *gee_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* GEE_H */
