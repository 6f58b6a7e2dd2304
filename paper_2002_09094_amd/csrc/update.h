// Argument blocks and launch wrappers of the update step: validation, the
// objects' term-major view, the exact member sums (full and incremental),
// norms and the new mean-major means.
#pragma once

#include "kernels.h"

namespace ivf {

// ----------------------------------------------------------------- update side
struct ObjectView {
    const int64_t* x_ptr;
    const int32_t* x_idx;
    const float* x_val;
    int64_t n, d, nnz;
};

// Validation of the object set: raises bits of Counters::error_flags.
hipError_t launch_validate_objects(const ObjectView& x, Counters* cnt, hipStream_t s);
// Validation of caller-given mean-major means.
hipError_t launch_validate_means(const int64_t* ptr, const int32_t* idx, const double* val,
                                 int32_t k, int64_t d, int64_t nnz, Counters* cnt,
                                 hipStream_t s);
// rowid[e] = object of entry e.
hipError_t launch_row_ids(const int64_t* ptr, int64_t n, int32_t* rowid, hipStream_t s);
hipError_t launch_iota(uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_copy_keys(const int32_t* in, uint32_t* out, int64_t n, hipStream_t s);
// After sorting (term, position): term-major view of the objects, the object
// of every entry and its (term, FP32 value bits).
hipError_t launch_build_xt(const uint32_t* sorted_terms, const uint32_t* sorted_pos,
                           const int32_t* rowid, const float* x_val, int64_t nnz,
                           int32_t* xt_obj, uint2* xt_tv, hipStream_t s);
// Per-term fixed-point scale: every member sum of term t is exact in units of
// 2^shift[t] unless the term's values span too wide a range (then rounded).
hipError_t launch_term_shift(const int32_t* x_idx, const float* x_val, int64_t nnz, int64_t d,
                             int32_t* emin, int32_t* emax, int32_t* count, int16_t* shift,
                             Counters* cnt, hipStream_t s);

// Segments per work item of the update's norm pass, and the most items any
// update of k clusters over nnz object entries can have.
constexpr int64_t kNormChunk = 4096;
inline int64_t norm_item_bound(int64_t k, int64_t nnz) { return k + nnz / kNormChunk + 1; }

struct UpdateArgs {
    int64_t n, d, nnz;
    int32_t k;
    const int32_t* assign;
    const int32_t* xt_obj;
    const uint2* xt_tv;     // (term, FP32 value bits) per term-major entry
    const int16_t* shift;
    // sort buffers (nnz)
    uint32_t* keys;
    uint32_t* keys_alt;
    uint2* pay;             // (term, value) of the entries in cluster order
    // segments (nnz capacity)
    uint32_t* flag;
    uint32_t* segpos;
    unsigned long long* seg_acc;
    int32_t* seg_j;
    int32_t* seg_t;
    // clusters
    int64_t* size;      // [k]
    int64_t* cstart;    // [k + 1]
    double* nrm;        // [k]
    double* objpart;    // [k]
    int64_t* newcnt;    // [k]
    int64_t* scal;      // device scalars: [0] valid entries, [1] segments
    int64_t* norm_items;  // [k + 1] norm work items per cluster, then their offsets
    double* norm_part;    // [2 * norm_item_bound(k, nnz)] per item: sum w^2, mu(old) . s
    // old means (mean-major) and new means
    const int64_t* old_ptr;
    const int32_t* old_idx;
    const double* old_val;
    int64_t* new_ptr;
    int64_t new_cap;    // entries the new-means buffers hold
    int32_t* new_idx;
    double* new_val;
    int32_t* new_row;
    Counters* cnt;
    void* tmp;
};

// Update, first half: group entries by cluster, exact per-(cluster, term)
// sums, sizes, norms, exact objective, new row counts and row pointers.
// launch_update_sums = launch_update_segments (cluster sizes, the sums as
// segments seg_j / seg_t / seg_acc, their count at scal[1]) followed by
// launch_update_norms (norms, objective shares and row pointers from the
// segments a.seg_* hold).
hipError_t launch_update_sums(UpdateArgs& a, hipStream_t s);
hipError_t launch_update_segments(UpdateArgs& a, hipStream_t s);
hipError_t launch_update_norms(UpdateArgs& a, hipStream_t s);

// Incremental form of launch_update_segments.  The table holds the sums of
// old_assign as (cluster, term, sum) in (cluster, term) order, tab_n entries,
// cstart its cluster starts.  The delta entries of the objects whose cluster
// changed (off: their scanned counts, `entries` in all) are reduced per
// (cluster, term) and merged into the table: the result, the sums of
// `assign`, is written to new_* (count at scal[1]) and equals what the full
// reduction gives.  tab_acc is modified in place.
struct DeltaArgs {
    const int64_t* x_ptr;
    const int32_t* x_idx;
    const float* x_val;
    int64_t n, d;
    int32_t k;
    const int32_t* assign;
    const int32_t* old_assign;
    const int64_t* off;          // [n + 1]
    int64_t entries;
    const int16_t* shift;
    int64_t* size;               // [k] in: the sizes of old_assign; out: those of assign
    int64_t* scal;
    // work buffers of >= entries elements
    uint32_t* keys;
    uint32_t* keys_alt;
    uint2* pay;
    uint2* pay_alt;
    uint32_t* flag;
    uint32_t* segpos;
    unsigned long long* dacc;    // delta segments: signed sums (two's complement)
    int32_t* dj;
    int32_t* dt;
    uint32_t* ins;
    uint32_t* ins_lb;
    uint32_t* ipos;
    // the table
    int64_t tab_n;
    const int64_t* cstart;       // [k + 1]
    const int32_t* tab_j;
    const int32_t* tab_t;
    unsigned long long* tab_acc;
    uint32_t* add;               // [tab_n + 1]
    int64_t* cs;                 // [tab_n + 1]
    int32_t* new_j;
    int32_t* new_t;
    unsigned long long* new_acc;
    void* tmp;
};
// Delta entry counts per object (off[i], then scanned in place: off[n] = total).
hipError_t launch_delta_count(const int64_t* x_ptr, int64_t n, const int32_t* assign,
                              const int32_t* old_assign, int32_t k, int64_t* off, void* tmp,
                              hipStream_t s);
hipError_t launch_delta_update(DeltaArgs& a, hipStream_t s);
// The first min(scal[1], cap) segments copied into a table.
hipError_t launch_copy_table(const int32_t* sj, const int32_t* st, const unsigned long long* sacc,
                             const int64_t* scal, int64_t cap, int32_t* tj, int32_t* tt,
                             unsigned long long* tacc, hipStream_t s);
// Update, second half: write the new mean-major means (after capacity check).
hipError_t launch_update_fill(UpdateArgs& a, hipStream_t s);
hipError_t launch_objective_exact(const double* objpart, int32_t k, double* out,
                                  hipStream_t s);
// Row ids of mean-major means (for caller-given means).
hipError_t launch_mean_rows(const int64_t* ptr, int32_t k, int32_t* row, hipStream_t s);

hipError_t launch_seed_assign(const int32_t* seeds, int32_t k, int64_t n, int32_t* assign,
                              hipStream_t s);

}  // namespace ivf
