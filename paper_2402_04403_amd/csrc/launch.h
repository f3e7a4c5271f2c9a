// Host-side launchers of the GEE kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gee {

// Per-vertex label record used by the edge pass: 1 byte (K <= 255), 2 bytes
// (K <= 65535) or 8 bytes (Laplacian: class + d^-1/2).
enum class Pack { U8, U16, LAP64 };

struct EmbedArgs {
    int64_t n = 0;
    int32_t K = 0;
    bool laplacian = false;
    bool weighted = false;
    Pack pack = Pack::U8;
    bool hot6 = false; // hot label table at 6 bits per slot (unit adjacency, 8-bit labels, K <= 63)
    bool atomic_updates = true; // push form: false = plain read-modify-write (diagnostic only)
    const int32_t *labels = nullptr;
    int32_t *err = nullptr;
    // workspace pieces
    uint64_t *counts = nullptr;  // [K+1]
    double *inv = nullptr;       // [K+1]
    void *lab = nullptr;         // [n] packed records
    double *deg = nullptr;       // [n] (Laplacian)
    float *Z = nullptr;
};

hipError_t launch_fill_u64(uint64_t *p, int64_t count, uint64_t value, hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t count, float value, hipStream_t s);
hipError_t launch_counts(const int32_t *labels, int64_t n, int32_t K, uint64_t *counts, void *packed,
                         Pack pack, int32_t *err, hipStream_t s);
hipError_t launch_weights(const uint64_t *counts, int32_t K, double *inv, hipStream_t s);
hipError_t launch_degrees_coo(int64_t n, int64_t ns, const int32_t *src, const int32_t *dst, const float *w,
                              double *deg, bool check_neg, int32_t *err, hipStream_t s);
hipError_t launch_degrees_csr(int64_t n, const int64_t *row_ptr, const float *val, int64_t nnz, double *deg,
                              bool check_neg, int32_t *err, hipStream_t s);
hipError_t launch_pack_lap(const int32_t *labels, int64_t n, int32_t K, const double *deg, uint64_t *lab,
                           hipStream_t s);
hipError_t launch_push(const EmbedArgs &a, int64_t ns, const int32_t *src, const int32_t *dst, const float *w,
                       hipStream_t s);
hipError_t launch_scale(const EmbedArgs &a, hipStream_t s);
hipError_t launch_seg_bounds(int64_t n, int64_t nnz, const int64_t *row_ptr, int64_t L, int64_t nseg,
                             int32_t *seg_i, int64_t *seg_e, hipStream_t s);
// LDS bytes one wavefront of the pull kernel uses for `rw` rows of K bins (wide_bins: the
// real-valued bins of the weighted and Laplacian versions).
size_t pull_wave_bytes(int32_t K, bool wide_bins, int rw);
// redo: [nseg] bytes of scratch, required for weighted adjacency (segments with a negative
// weight are summed again in FP64), else unused.
hipError_t launch_pull(const EmbedArgs &a, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                       const float *val, const void *hotlab, int64_t n_hot, const int32_t *seg_i,
                       const int64_t *seg_e, int64_t nseg, int rw, double *part, uint8_t *redo, hipStream_t s);
hipError_t launch_pack_hot(const EmbedArgs &a, const int32_t *hot_ids, int64_t n_hot, void *hotlab, hipStream_t s);
hipError_t launch_merge(const EmbedArgs &a, const int64_t *row_ptr, const int32_t *seg_i, const int64_t *seg_e,
                        int64_t nseg, const double *part, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);

// Batched pull: one group of up to 64 label vectors (any mix of adjacency and
// Laplacian) whose column blocks are contiguous in Z, embedded in one pass of the
// CSR. Group column f in [0, KT) is class f - coff_b + 1 of the vector b with
// coff_b <= f < coff_b + K_b, and Z column zcol + f.
constexpr int kGroupMax = 64;
constexpr int kBatchMaxKT = 4096;               // classes of one group: KT FP64 bins per wavefront
constexpr size_t kBatchLdsBytes = 160 * 1024;   // LDS of one block: column scales + bins of each wavefront
struct GroupDesc {
    int G = 0;                  // vectors in the group
    int Gs = 0;                 // label-matrix row stride (G + 1 rounded up to 8, at most 64)
    int KT = 0;                 // sum of K over the group
    int32_t vec[kGroupMax];     // index of each vector in the caller's batch
    int32_t K[kGroupMax];       // classes of each vector
    int32_t coff[kGroupMax];    // first group column of each vector
    int64_t zoff[kGroupMax];    // first Z column of each vector
    int64_t inv_off[kGroupMax]; // offset of each vector's class counts in the batch's counts array
    uint8_t lap[kGroupMax];     // 1: Laplacian version
};
struct GroupArgs {
    int64_t n = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const float *val = nullptr;
    int64_t n_hot = 0;
    const void *labmat = nullptr; // [(n + 1) * Gs] labels, 8-bit (u8) or 16-bit
    const void *labhot = nullptr; // [n_hot * Gs]
    bool u8 = false;              // every vector of the group has K <= 255
    int Gs = 0, KT = 0;
    const float *rsd = nullptr;       // [n], Laplacian groups
    const float *rsdhot = nullptr;    // [n_hot], Laplacian groups
    const uint32_t *vmeta = nullptr;  // [64]
    const double *cscale = nullptr;   // [KT]
    const int32_t *seg_i = nullptr;
    const int64_t *seg_e = nullptr;
    int64_t nseg = 0;
    float *Z = nullptr;
    int64_t ldz = 0, zcol = 0;
    double *part = nullptr;
    int32_t *err = nullptr;
    bool lap = false; // the group holds Laplacian vectors
};
int batch_waves_per_block(int KT); // wavefronts whose bins fit one block's LDS beside the scale table
size_t batch_lds_bytes(int KT, int nw);
hipError_t launch_pack_group(const int32_t *labels, int64_t n, const GroupDesc &d, void *labmat, bool u8, int32_t *err,
                             hipStream_t s);
// Class counts of every vector of a group (added to counts, which start at zero); each
// vector's K + 1 counts at its inv_off.
hipError_t launch_counts_group(const int32_t *labels, int64_t n, const GroupDesc &d, uint64_t *counts, int32_t *err,
                               hipStream_t s);
hipError_t launch_pack_group_hot(const int32_t *hot_ids, int64_t n_hot, int64_t n, int row_bytes, const void *labmat,
                                 void *labhot, const float *rsd, float *rsdhot, int32_t *err, hipStream_t s);
hipError_t launch_group_cols(const uint64_t *counts_all, const GroupDesc &d, double *cscale, uint32_t *vmeta,
                             hipStream_t s);
hipError_t launch_rsd(const double *deg, int64_t n, float *rsd, hipStream_t s);
hipError_t launch_pull_group(const GroupArgs &g, hipStream_t s);

// Sorting and scanning pieces of the CSR build, shared by the propagation-blocked layout
size_t radix_scratch_bytes(int64_t N, int64_t scan_n, size_t *hist_bytes, size_t *offs_bytes, size_t *part_bytes);
// Stable LSD sort of N keys on bits [lo, hi) in 8-bit digits, ping-ponging between the two
// buffers; *result is the buffer that holds the sorted keys.
hipError_t radix_sort_bits(uint64_t *keys0, uint64_t *keys1, int64_t N, int lo, int hi, uint32_t *hist,
                           int64_t *offs, int64_t *scan_part, uint64_t **result, hipStream_t s);
// The same with a float carried along with each key.
hipError_t radix_sort_bits_kv(uint64_t *keys0, uint64_t *keys1, float *vals0, float *vals1, int64_t N, int lo, int hi,
                              uint32_t *hist, int64_t *offs, int64_t *scan_part, uint64_t **rkeys, float **rvals,
                              hipStream_t s);
hipError_t max_scan_i64(const int64_t *in, int64_t N, int64_t *out, int64_t *scan_part, hipStream_t s); // inclusive
hipError_t launch_fill_i64(int64_t *p, int64_t count, int64_t value, hipStream_t s);

// Propagation-blocked pull (unit-weight adjacency): entries of the CSR in column-block
// order, 256-row blocks, 2^21-vertex column blocks, then up to 32 blocks ("tier slices")
// of 2^17 hot slots each whose labels are read from LDS.
constexpr int kPbRowBits = 8;
constexpr int kPbColBits = 21;
constexpr int kPbMaxK = 255;                       // 8-bit labels; above 128 classes the bins are 16-bit (or two passes)
constexpr int kPbSliceBits = 17;                   // tier slice: 128 KB of 8-bit labels
constexpr int64_t kPbSlice = (int64_t)1 << kPbSliceBits;
constexpr int kPbMaxSlices = 512;                  // tier slots <= 2^26
constexpr int64_t kPbMaxNnz = (int64_t)UINT32_MAX - 64; // cell lengths and word prefixes are 32-bit
struct PbLayout {
    int64_t n_rb = 0;
    int32_t n_vcb = 0; // vertex column blocks
    int32_t n_sl = 0;  // tier slices
    int32_t n_cb = 0;  // n_vcb + n_sl
    int64_t cells = 0;
};
PbLayout pb_layout(int64_t n, int64_t n_lds);
constexpr int kPbF32Terms = 128; // a weighted row block sums in FP32 when its rows have at most this many entries
// meta[4] of a weighted layout whose weights are not all multiples of one power of two
// small enough for exact 32-bit sums
constexpr int64_t kPbNoGrid = -((int64_t)1 << 62);
size_t pb_build_scratch(int64_t n, int64_t nnz, int64_t n_lds, bool weighted, bool laplacian);
// val (CSR weights) null for unit weights. vl and rb_flag are written for a weighted or a
// Laplacian layout (vl: w, or w d_v^-1/2), rsd for a Laplacian layout.
hipError_t launch_pb_build(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const float *val,
                           bool laplacian, const int32_t *hot_ids, int64_t n_hot, int64_t n_lds, int32_t *colc,
                           uint8_t *ul, int64_t *cell_start, uint32_t *cell_count, uint32_t *cell_word,
                           int32_t *lds_ids, float *vl, uint8_t *rb_flag, float *rsd, int64_t *meta, void *ws,
                           int32_t *err, hipStream_t s);
// tab: per-call scratch of (n_lds rounded up to 16) bytes.
// A layout whose fingerprint (meta) disagrees with n, nnz, n_lds and its kind (0 unit
// adjacency, 1 weighted adjacency, 2 Laplacian) raises GEE_EVERTEX in err and is not read.
hipError_t launch_pb_gather(int64_t n, int64_t nnz, const PbLayout &L, int64_t n_lds, const int64_t *cell_start,
                            const uint32_t *cell_count, const int32_t *colc, const int32_t *lds_ids,
                            const int64_t *meta, int kind, const uint8_t *lab, uint8_t *tab, uint8_t *yv,
                            int32_t *err, hipStream_t s);
// slice_entries [ceil(n_slots / 2^17)]: entries whose column is a hot slot of that slice.
hipError_t launch_pb_slice_entries(int64_t n_slots, const int32_t *hot_ids, const int64_t *row_ptr,
                                  int64_t *slice_entries, hipStream_t s);
// ul and yv: 4-byte aligned, readable up to nnz + 32 (the gap before the tier included).
// A cell outside the layout's nnz + 15 entries is read as empty and raises GEE_EVERTEX.
// vl and rb_flag: a weighted or Laplacian layout's values and row-block flags, else null;
// rsd: a Laplacian layout's d^-1/2, else null.
hipError_t launch_pb_rows(int64_t n, int64_t nnz, int32_t K, const PbLayout &L, const int64_t *cell_start,
                          const uint32_t *cell_count, const uint32_t *cell_word, const uint8_t *ul, const uint8_t *yv,
                          const float *vl, const uint8_t *rb_flag, const float *rsd, const int64_t *meta,
                          int64_t n_lds, const double *inv, float *Z, int32_t *err, hipStream_t s);

// Labels from an embedding: out[u] = 1 + argmax_k Z[u][k] (first maximum; 0 for a row
// with no positive entry); changed (nullable) is set to the number of rows where out
// differs from prev (prev nullable).
hipError_t launch_argmax(int64_t n, int32_t K, int64_t ldz, const float *Z, const int32_t *prev, int32_t *out,
                         uint64_t *changed, hipStream_t s);

// CSR build
struct CsrBuildWs {
    uint64_t *keys[2];
    float *vals[2];
    uint32_t *hist;     // [256 * nblocks]
    int64_t *offs;      // [256 * nblocks]
    int64_t *scan_part; // scan partials
    int64_t *rowlast;   // [n]
    int64_t *vtmp[2];   // [n] each: hot-vertex selection scratch
    uint64_t *hkeys[2]; // [n_hot] each: hot vertices keyed by degree bucket
    int64_t *hot_hist;  // degree histogram
    int64_t *hot_par;   // threshold, quota
};
size_t csr_build_layout(int64_t n, int64_t s, bool weighted, int64_t n_hot, char *base, CsrBuildWs *out);
hipError_t launch_csr_build(int64_t n, int64_t ns, const int32_t *src, const int32_t *dst, const float *w,
                            int64_t n_hot, int64_t *row_ptr, int32_t *col, float *val, int32_t *hot_ids,
                            const CsrBuildWs &ws, int32_t *err, hipStream_t s);

} // namespace gee
