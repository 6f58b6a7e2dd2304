// Argument blocks and launch wrappers of the assignment walk, its merge and
// FP64 re-score, IVFD, and the inverted-file rebuild the walk reads.
#pragma once

#include "ivf_internal.h"

namespace ivf {

struct WalkArgs {
    const int64_t* x_ptr;
    const int32_t* x_idx;
    const float* x_val;
    int64_t n;
    const SliceDesc* desc;    // [d * R]: per (term, range) slice, sparse or dense
    const void* post;         // uint2 {cluster, f32} or uint32 {local cluster | 16-bit value}
    const void* slab;         // dense slices: float or 16-bit values, zeros for absent clusters
    int32_t k, k_r, R, chunk, tile_stride;
    int64_t items_per_range;  // ceil(n / chunk)
    Counters* cnt;
    RangeRec* rec;            // [R * n], range-major: record (i, r) at r * n + i
};

struct MergeArgs {
    const int64_t* x_ptr;
    int64_t n;
    int32_t R;
    int32_t valtype, certify, force_rescore;
    double fixed_scale;       // > 0: the records hold fixed-point sums (IVFD) of this scale
    double vmax;              // largest object value (the certificate's absolute terms)
    const RangeRec* rec;      // [R * n] range-major: record (i, r) at r * n + i
    const int32_t* prev;
    int32_t* assign;
    double* rho;
    float* best;
    int32_t* best_id;
    float* second;
    uint8_t* flags;
    int32_t* rescore_list;
    Counters* cnt;
};

struct RescoreArgs {
    WalkArgs w;               // the walk's view of the objects and the inverted file
    const int64_t* mm_ptr;    // [k + 1] the walk's means, mean-major FP64
    const int32_t* mm_idx;
    const double* mm_val;
    int32_t valtype;
    double fixed_scale;       // > 0: `best` is a fixed-point sum (IVFD) of this scale
    double vmax;              // largest object value (the certificate's absolute terms)
    const RangeRec* rec;      // the walk's range records, [w.R * n] range-major (null: re-walk every range)
    const int32_t* rescore_list;
    const int32_t* prev;
    int32_t* assign;
    double* rho;
    const float* best;
    const int32_t* best_id;
    Counters* cnt;
};

hipError_t launch_clear_counters(Counters* c, hipStream_t s);
hipError_t walk_set_lds_limit(int lds_bytes);
// The walk kernel a plan launches: FP32 ranges of up to 1,024 clusters take
// the register walk (for a batch: every instance within tile_stride).
const void* walk_kernel_ptr(int valtype, int32_t k_r);
const void* walk_batch_kernel_ptr(int valtype, int32_t tile_stride);
// Walk of many instances in one persistent launch (args, item_off: device;
// work: a device counter the launch resets and the waves claim items from).
hipError_t launch_walk_batch(const WalkArgs* args, const int64_t* item_off, int32_t count,
                             int32_t tile_stride, int valtype, int waves, int grid,
                             unsigned long long* work, hipStream_t s);
hipError_t launch_walk(const WalkArgs& a, int valtype, int waves, int lds_bytes, int grid,
                       hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
// FP64 re-score of the queued objects: `waves` waves per workgroup, each with
// its own tile of w.tile_stride floats.
hipError_t launch_rescore(const RescoreArgs& a, int waves, int grid, hipStream_t s);
const void* rescore_kernel_ptr(int valtype);
hipError_t launch_objective(const double* rho, const int32_t* assign, const int32_t* prev,
                            int64_t n, double* part, int nblocks, double* out, Counters* cnt,
                            hipStream_t s);

// ------------------------------------------------------------------ IVFD walk
// The assignment with the objects inverted: one workgroup per range of n_r
// objects walks every mean over the range's slice of the objects' inverted
// file and keeps the objects' running (best, cluster, second) in registers.
struct IvfdArgs {
    const uint32_t* optr;     // [R * d + 1] slice bounds, range-major then term
    const uint2* opost;       // {object - range start, FP32 value bits}
    const int64_t* mm_ptr;    // [k + 1] the means, mean-major FP64
    const int32_t* mm_idx;
    const double* mm_val;
    int64_t n, d;
    int32_t k, R, n_r;        // n_r in {4096, 8192, 16384}
    int32_t B;                // blocks of consecutive means; workgroup = (range, block)
    float scale, inv_scale;   // fixed-point scale 2^F of the products, and 2^-F
    RangeRec* rec;            // [B * n], block-major: best, id, second (m: launch_ivfd_overlap)
    unsigned long long* walked;   // entries walked, added
};

int ivfd_lds_bytes(int32_t n_r);
// Objects' inverted file in (range, term, object) order from the row ids:
// keys/vals/keys_alt/vals_alt/tmp are sort scratch of nnz entries, iota the
// identity permutation, nkeys = R * d.
hipError_t launch_ivfd_build(const int32_t* rowid, const int32_t* x_idx, const float* x_val,
                             int64_t nnz, int32_t n_r, int64_t d, int64_t nkeys, uint32_t* keys,
                             uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                             const uint32_t* iota, void* tmp, uint32_t* optr, uint2* post,
                             hipStream_t s);
hipError_t launch_ivfd_walk(const IvfdArgs& a, hipStream_t s);
// rec[i * B + b].m = the object's share of M for b == 0, else 0.
hipError_t launch_ivfd_overlap(const int64_t* x_ptr, const int32_t* x_idx, int64_t n, int32_t B,
                               const int64_t* ivf_ptr, RangeRec* rec, hipStream_t s);
// Largest L2 norm (FP64) of the rows of a CSR matrix with `rows` rows, as
// double bits atomically maxed into *out (which the caller zeroes).
hipError_t launch_max_row_norm(const int64_t* ptr, const float* val32, const double* val64,
                               int64_t rows, unsigned long long* out, hipStream_t s);

// ------------------------------------------------ inverted-file rebuild
struct IvfArgs {
    int64_t d, nnzM;          // nnzM: entries, or their capacity if nnz_dev is set
    const int64_t* nnz_dev;   // device-side entry count (nullable)
    int32_t k, k_r, R, valtype;
    float dense_threshold;
    const int32_t* mm_idx;
    const double* mm_val;
    const int32_t* mm_row;
    uint32_t* keys;
    uint32_t* keys_alt;
    uint2* pay;          // (cluster, FP32 value bits) per entry, sorted with the keys
    uint2* pay_alt;
    int64_t* ivf_ptr;    // [d + 1]
    SliceDesc* desc;     // [d * R]
    int64_t* dsz;        // [d * R + 1] dense slab sizes, then their offsets (scanned)
    void* slab;          // dense slabs (sized by the first phase)
    int32_t* cid;        // [nnzM]
    void* post;          // [nnzM] uint2 or uint32
    void* tmp;
};

// Inverted-file rebuild, phase 1: stable sort of the mean entries by term
// with their cluster and value as payload, lists in ascending cluster order
// with the stored-precision values, slice descriptors and the scanned
// dense-slab offsets (total at dsz[d * R]).  keys/keys_alt and pay/pay_alt
// hold at least nnzM entries.
hipError_t launch_build_ivf(IvfArgs& a, hipStream_t s);
// Phase 2: dense slabs filled (the array holds slab_cap elements; slices that
// do not fit stay sparse), descriptors of dense slices pointed at them.
hipError_t launch_build_slabs(IvfArgs& a, int64_t slab_cap, hipStream_t s);

}  // namespace ivf
