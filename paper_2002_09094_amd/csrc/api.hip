// C ABI of the library (declared in include/ivf.h): handles, validation,
// planning, memory, the order of launches for one Lloyd iteration, and the
// batch of many instances replayed as captured HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ivf_internal.h"
#include "kernels.h"
#include "update.h"

using namespace ivf;

namespace {

constexpr int kObjBlocks = 1024;
thread_local std::string g_build_error;

template <typename T>
hipError_t dalloc(T** p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    return hipMalloc(reinterpret_cast<void**>(p), (size_t)count * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(reinterpret_cast<void*>(p));
    p = nullptr;
}

// Transient buffers of the update and of the inverted-file rebuild.  A batch
// shares one set, sized for its largest instance.
struct Scratch {
    int64_t sort_cap = 0;   // entries of the sort buffers
    int64_t seg_cap = 0;    // entries of the segment buffers
    int64_t scan_need = 0;  // largest scan any user runs
    uint32_t *keys = nullptr, *vals = nullptr, *keys_alt = nullptr, *vals_alt = nullptr;
    uint32_t* iota = nullptr;
    uint32_t *flag = nullptr, *segpos = nullptr;
    unsigned long long* seg_acc = nullptr;
    uint2* pay = nullptr;   // update: (term, value) payload sorted by cluster
    int32_t *seg_j = nullptr, *seg_t = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;

    void release() {
        dfree(keys); dfree(vals); dfree(keys_alt); dfree(vals_alt); dfree(iota);
        dfree(flag); dfree(segpos); dfree(seg_acc); dfree(seg_j); dfree(seg_t); dfree(pay);
        if (tmp) (void)hipFree(tmp);
        tmp = nullptr;
        sort_cap = seg_cap = 0;
        tmp_bytes = 0;
    }

    hipError_t ensure(int64_t sort_need, int64_t seg_need, int64_t scan, hipStream_t s) {
        scan_need = std::max(scan_need, scan);
        if (sort_need > sort_cap) {
            const int64_t cap = std::max<int64_t>(sort_need, sort_cap + sort_cap / 4);
            dfree(keys); dfree(vals); dfree(keys_alt); dfree(vals_alt); dfree(iota);
            sort_cap = 0;
            hipError_t e;
            if ((e = dalloc(&keys, cap)) != hipSuccess) return e;
            if ((e = dalloc(&vals, cap)) != hipSuccess) return e;
            if ((e = dalloc(&keys_alt, cap)) != hipSuccess) return e;
            if ((e = dalloc(&vals_alt, cap)) != hipSuccess) return e;
            if ((e = dalloc(&iota, cap)) != hipSuccess) return e;
            if ((e = launch_iota(iota, cap, s)) != hipSuccess) return e;
            sort_cap = cap;
        }
        if (seg_need > seg_cap) {
            dfree(flag); dfree(segpos); dfree(seg_acc); dfree(seg_j); dfree(seg_t); dfree(pay);
            seg_cap = 0;
            hipError_t e;
            if ((e = dalloc(&flag, seg_need)) != hipSuccess) return e;
            if ((e = dalloc(&segpos, seg_need)) != hipSuccess) return e;
            if ((e = dalloc(&seg_acc, seg_need)) != hipSuccess) return e;
            if ((e = dalloc(&seg_j, seg_need)) != hipSuccess) return e;
            if ((e = dalloc(&seg_t, seg_need)) != hipSuccess) return e;
            if ((e = dalloc(&pay, seg_need)) != hipSuccess) return e;
            seg_cap = seg_need;
        }
        const size_t need = std::max(radix_tmp_bytes(std::max<int64_t>(sort_cap, 1)),
                                     scan_tmp_bytes(std::max<int64_t>(
                                         std::max(sort_cap, seg_cap), scan_need)));
        if (need > tmp_bytes) {
            if (tmp) (void)hipFree(tmp);
            tmp = nullptr;
            tmp_bytes = 0;
            hipError_t e = hipMalloc(&tmp, need);
            if (e != hipSuccess) return e;
            tmp_bytes = need;
        }
        return hipSuccess;
    }
};

// Term-major view of one object set and its per-term fixed-point scales;
// handles clustering the same set share one.
struct ObjView {
    const int64_t* x_ptr = nullptr;
    const int32_t* x_idx = nullptr;
    const float* x_val = nullptr;
    int64_t n = 0, d = 0, nnz = 0;
    int32_t* xt_obj = nullptr;
    uint2* xt_tv = nullptr;
    int16_t* shift = nullptr;
    int64_t inexact = 0;
    // IVFD: the objects' inverted file, range-major (built on first use)
    int32_t o_nr = 0;           // objects per range, 0 = not built
    int64_t o_R = 0;            // ranges
    uint32_t* optr = nullptr;   // [o_R * d + 1]
    uint2* opost = nullptr;     // [nnz]
    double o_maxnorm = 0.0;     // largest object L2 norm
    double vmax = 0.0;          // largest object value
    int64_t nmax = 0;           // longest object row

    void release() { dfree(xt_obj); dfree(xt_tv); dfree(shift); dfree(optr); dfree(opost); }
};

}  // namespace

struct ivf_handle {
    int64_t n = 0, d = 0, nnz = 0;
    int32_t k = 0;
    ivf_options opt{};
    hipStream_t stream = nullptr;
    Plan plan;
    int device = 0, cus = 0;
    int walk_grid = 0, rescore_grid = 0, rescore_waves = 1;
    ObjView* ov = nullptr;
    bool owns_ov = false;
    Scratch* sc = nullptr;
    bool owns_sc = false;
    // capacities fixed (no host synchronisation, no allocation): graph capture
    bool fixed = false;
    // means, mean-major FP64, double-buffered
    int cur = 0;
    bool has_means = false;
    bool nnzM_known = true;    // false while the count lives only on the device
    double mmax = 1.0;         // largest mean value any current mean may hold
    int64_t nnzM = 0;
    int64_t mm_cap[2] = {0, 0};
    int64_t* mm_ptr[2] = {nullptr, nullptr};
    int32_t* mm_idx[2] = {nullptr, nullptr};
    double* mm_val[2] = {nullptr, nullptr};
    int32_t* mm_row[2] = {nullptr, nullptr};
    // inverted file
    int64_t ivf_cap = 0;
    int64_t* ivf_ptr = nullptr;
    SliceDesc* desc = nullptr;
    int64_t* dsz = nullptr;
    int32_t* cid = nullptr;
    void* post = nullptr;
    void* slab = nullptr;
    int64_t slab_cap = 0;      // elements
    int64_t slab_need = 0;     // most elements any rebuild asked for
    // clusters
    int64_t *size = nullptr, *cstart = nullptr, *newcnt = nullptr, *scal = nullptr;
    double *nrm = nullptr, *objpart = nullptr;
    int64_t* norm_items = nullptr;
    double* norm_part = nullptr;
    // assignment
    RangeRec* rec = nullptr;
    RangeRec* ivfd_rec = nullptr;   // IVFD: one record per object and block of means
    int64_t ivfd_rec_cap = 0;
    int32_t* prev = nullptr;
    int32_t* seed_assign = nullptr;
    double* rho = nullptr;
    float *best = nullptr, *second = nullptr;
    int32_t* best_id = nullptr;
    uint8_t* flags = nullptr;
    int32_t* rescore_list = nullptr;
    double* part = nullptr;
    double* dscal = nullptr;   // [0] objective, [1] exact objective
    Counters* cnt = nullptr;
    // incremental update: the exact member sums of tab_assign, in (cluster,
    // term) order (table tc; the other is the next update's output), and the
    // merge's work arrays, sized with the tables
    bool tab_valid = false;
    int tc = 0;
    int64_t tab_n = 0;
    int64_t tab_cap[2] = {0, 0};
    int32_t* tab_j[2] = {nullptr, nullptr};
    int32_t* tab_t[2] = {nullptr, nullptr};
    unsigned long long* tab_acc[2] = {nullptr, nullptr};
    int64_t merge_cap = 0;
    uint32_t* merge_add = nullptr;
    int64_t* merge_cs = nullptr;
    int32_t* tab_assign = nullptr;
    int64_t* delta_off = nullptr;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    std::string err;
};

namespace {

ivf_status fail(ivf_handle* h, ivf_status st, const std::string& msg) {
    if (h) h->err = msg;
    else g_build_error = msg;
    return st;
}

#define HIPCHK(h, call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail((h), e_ == hipErrorOutOfMemory ? IVF_ERR_OOM : IVF_ERR_HIP,      \
                        std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

void free_handle(ivf_handle* h) {
    if (h->owns_ov && h->ov) { h->ov->release(); delete h->ov; }
    h->ov = nullptr;
    if (h->owns_sc && h->sc) { h->sc->release(); delete h->sc; }
    h->sc = nullptr;
    for (int b = 0; b < 2; ++b) {
        dfree(h->mm_ptr[b]); dfree(h->mm_idx[b]); dfree(h->mm_val[b]); dfree(h->mm_row[b]);
    }
    dfree(h->ivf_ptr); dfree(h->desc); dfree(h->dsz); dfree(h->cid);
    if (h->post) (void)hipFree(h->post);
    h->post = nullptr;
    if (h->slab) (void)hipFree(h->slab);
    h->slab = nullptr;
    dfree(h->size); dfree(h->cstart); dfree(h->newcnt); dfree(h->scal);
    dfree(h->nrm); dfree(h->objpart); dfree(h->norm_items); dfree(h->norm_part);
    dfree(h->rec); dfree(h->ivfd_rec); dfree(h->prev); dfree(h->seed_assign); dfree(h->rho); dfree(h->best);
    dfree(h->second); dfree(h->best_id); dfree(h->flags); dfree(h->rescore_list);
    dfree(h->part); dfree(h->dscal); dfree(h->cnt);
    for (int b = 0; b < 2; ++b) { dfree(h->tab_j[b]); dfree(h->tab_t[b]); dfree(h->tab_acc[b]); }
    dfree(h->merge_add); dfree(h->merge_cs); dfree(h->tab_assign); dfree(h->delta_off);
    for (auto& e : h->ev)
        if (e) { (void)hipEventDestroy(e); e = nullptr; }
}

// Scratch for sorts of sort_need entries: the u32 sort buffers, and the
// segment arrays (whose payload pair the inverted-file rebuild sorts with) for
// max(object entries, sort_need).
ivf_status ensure_scratch(ivf_handle* h, int64_t sort_need) {
    const int64_t scan = std::max<int64_t>((int64_t)h->k + 1, h->d * (int64_t)h->plan.R + 1);
    const int64_t seg_need = std::max<int64_t>(h->nnz, sort_need);
    if (h->fixed) {
        if (sort_need <= h->sc->sort_cap && seg_need <= h->sc->seg_cap && scan <= h->sc->scan_need)
            return IVF_OK;
        return fail(h, IVF_ERR_CAPACITY, "scratch exceeds the fixed capacity");
    }
    HIPCHK(h, h->sc->ensure(sort_need, seg_need, scan, h->stream));
    return IVF_OK;
}

// Mean-major buffer `b` grown to hold `need` entries; the first `keep`
// entries are carried over (0: the content is about to be overwritten).
ivf_status ensure_mm(ivf_handle* h, int b, int64_t need, int64_t keep = 0) {
    if (need <= h->mm_cap[b]) return IVF_OK;
    if (h->fixed) return fail(h, IVF_ERR_CAPACITY, "means exceed the fixed capacity");
    const int64_t cap = std::max<int64_t>(need, h->mm_cap[b] + h->mm_cap[b] / 4);
    keep = std::min(keep, h->mm_cap[b]);
    int32_t* idx = nullptr;
    double* val = nullptr;
    int32_t* row = nullptr;
    hipError_t e = dalloc(&idx, cap);
    if (e == hipSuccess) e = dalloc(&val, cap);
    if (e == hipSuccess) e = dalloc(&row, cap);
    if (e == hipSuccess && keep > 0) {
        e = hipMemcpyAsync(idx, h->mm_idx[b], sizeof(int32_t) * (size_t)keep,
                           hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(val, h->mm_val[b], sizeof(double) * (size_t)keep,
                               hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(row, h->mm_row[b], sizeof(int32_t) * (size_t)keep,
                               hipMemcpyDeviceToDevice, h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);   // copies done before the frees
    if (e != hipSuccess) {
        dfree(idx); dfree(val); dfree(row);
        return fail(h, e == hipErrorOutOfMemory ? IVF_ERR_OOM : IVF_ERR_HIP,
                    std::string("growing the means: ") + hipGetErrorString(e));
    }
    dfree(h->mm_idx[b]); dfree(h->mm_val[b]); dfree(h->mm_row[b]);
    h->mm_idx[b] = idx;
    h->mm_val[b] = val;
    h->mm_row[b] = row;
    h->mm_cap[b] = cap;
    return IVF_OK;
}

ivf_status ensure_ivf(ivf_handle* h, int64_t need) {
    if (need > h->ivf_cap) {
        if (h->fixed) return fail(h, IVF_ERR_CAPACITY, "inverted file exceeds the fixed capacity");
        const int64_t cap = std::max<int64_t>(need, h->ivf_cap + h->ivf_cap / 4);
        dfree(h->cid);
        if (h->post) (void)hipFree(h->post);
        h->post = nullptr;
        h->ivf_cap = 0;
        HIPCHK(h, dalloc(&h->cid, cap));
        HIPCHK(h, hipMalloc(&h->post, (size_t)std::max<int64_t>(cap, 1) * 8));
        h->ivf_cap = cap;
    }
    return ensure_scratch(h, need);
}

ivf_status ensure_slab(ivf_handle* h, int64_t elems) {
    // slices beyond the cap stay sparse (descriptors address slabs with 31 bits)
    elems = std::min(elems, kMaxSlabElems);
    if (elems <= h->slab_cap || h->fixed) return IVF_OK;   // fixed: misfits stay sparse
    if (h->slab) (void)hipFree(h->slab);
    h->slab = nullptr;
    h->slab_cap = 0;
    const int64_t cap = std::min(elems + elems / 4, kMaxSlabElems);
    HIPCHK(h, hipMalloc(&h->slab, (size_t)cap * (h->opt.valtype == IVF_VAL_F32 ? 4 : 2)));
    h->slab_cap = cap;
    return IVF_OK;
}

// Table b of the incremental update grown to `need` entries (its content is
// about to be overwritten), and the merge arrays to cover a table of `need`.
ivf_status ensure_tab(ivf_handle* h, int b, int64_t need) {
    need = std::max<int64_t>(need, 1);
    if (need > h->tab_cap[b]) {
        const int64_t cap = std::max<int64_t>(need, h->tab_cap[b] + h->tab_cap[b] / 4);
        dfree(h->tab_j[b]); dfree(h->tab_t[b]); dfree(h->tab_acc[b]);
        h->tab_cap[b] = 0;
        HIPCHK(h, dalloc(&h->tab_j[b], cap));
        HIPCHK(h, dalloc(&h->tab_t[b], cap));
        HIPCHK(h, dalloc(&h->tab_acc[b], cap));
        h->tab_cap[b] = cap;
    }
    if (need + 1 > h->merge_cap) {
        const int64_t cap = std::max<int64_t>(need + 1, h->merge_cap + h->merge_cap / 4);
        dfree(h->merge_add); dfree(h->merge_cs);
        h->merge_cap = 0;
        HIPCHK(h, dalloc(&h->merge_add, cap));
        HIPCHK(h, dalloc(&h->merge_cs, cap));
        h->merge_cap = cap;
    }
    return IVF_OK;
}

ivf_status read_errors(ivf_handle* h, const char* what, Counters* out = nullptr) {
    Counters c;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
    if (out) *out = c;
    const unsigned long long f = c.error_flags;
    if (!f) return IVF_OK;
    std::string m = std::string(what) + ": ";
    if (f & kOverflow) return fail(h, IVF_ERR_CAPACITY, m + "new means exceed the fixed capacity");
    if (f & kBadPtr) return fail(h, IVF_ERR_ARG, m + "row pointers inconsistent with sizes");
    if (f & kBadIndex) return fail(h, IVF_ERR_UNSORTED, m + "term id outside [0, d)");
    if (f & kBadOrder) return fail(h, IVF_ERR_UNSORTED, m + "term ids not strictly ascending");
    if (f & kNonFinite) return fail(h, IVF_ERR_NONFINITE, m + "non-finite value");
    return fail(h, IVF_ERR_NEGATIVE, m + "value <= 0");
}

// FP32 scores must stay finite: every score is at most (longest row) x
// (largest object value) x (largest mean value), kept below 2^120; FP16 mean
// values must fit FP16's range.
ivf_status check_value_range(ivf_handle* h, double mmax) {
    const double top = (double)std::max<int64_t>(h->ov->nmax, 1) * h->ov->vmax * mmax;
    if (!(top < 0x1p120) || !(mmax < 0x1p120))
        return fail(h, IVF_ERR_CAPACITY,
                    "values too large: FP32 scores could overflow (rows x largest object value "
                    "x largest mean value >= 2^120)");
    if (h->opt.valtype == IVF_VAL_F16 && mmax >= 65504.0)
        return fail(h, IVF_ERR_CAPACITY, "a mean value is beyond FP16's range (>= 65504)");
    return IVF_OK;
}

IvfArgs ivf_args(ivf_handle* h, int b) {
    IvfArgs a{};
    a.d = h->d;
    a.k = h->k;
    a.k_r = h->plan.k_r;
    a.R = h->plan.R;
    a.valtype = h->opt.valtype;
    a.dense_threshold = h->opt.dense_threshold > 0.f ? h->opt.dense_threshold
                                                     : dense_default(h->opt.valtype, h->plan.k_r);
    a.mm_idx = h->mm_idx[b];
    a.mm_val = h->mm_val[b];
    a.mm_row = h->mm_row[b];
    a.keys = h->sc->keys;
    a.keys_alt = h->sc->keys_alt;
    a.pay = h->sc->pay;
    a.pay_alt = reinterpret_cast<uint2*>(h->sc->seg_acc);
    a.ivf_ptr = h->ivf_ptr;
    a.desc = h->desc;
    a.dsz = h->dsz;
    a.cid = h->cid;
    a.post = h->post;
    a.slab = h->slab;
    a.tmp = h->sc->tmp;
    return a;
}

// Inverted file from mean-major buffer `b`.  With nnz_dev the entry count is
// read on the device (capacity-bounded, no host synchronisation).
ivf_status rebuild_ivf(ivf_handle* h, int b, int64_t nnzM, const int64_t* nnz_dev) {
    if (nnzM >= ((int64_t)1 << 31) ||
        (nnz_dev && std::max(h->mm_cap[0], h->mm_cap[1]) >= ((int64_t)1 << 31)))
        return fail(h, IVF_ERR_CAPACITY, "the means hold 2^31 or more entries");
    ivf_status st = ensure_ivf(h, nnzM);
    if (st != IVF_OK) return st;
    IvfArgs a = ivf_args(h, b);
    a.nnzM = nnz_dev ? std::min(h->ivf_cap, h->mm_cap[b]) : nnzM;
    a.nnz_dev = nnz_dev;
    HIPCHK(h, launch_build_ivf(a, h->stream));
    if (!h->fixed) {
        // size the dense slabs (the scanned total) before filling them
        int64_t elems = 0;
        HIPCHK(h, hipMemcpyAsync(&elems, h->dsz + h->d * h->plan.R, sizeof(int64_t),
                                 hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        h->slab_need = std::max(h->slab_need, elems);
        st = ensure_slab(h, elems);
        if (st != IVF_OK) return st;
        a.slab = h->slab;
    }
    HIPCHK(h, launch_build_slabs(a, h->slab_cap, h->stream));
    return IVF_OK;
}

// Update step from `assign`: new means into buffer 1 - cur, then the swap and
// the inverted-file rebuild.  In fixed mode nothing synchronises or allocates.
// clear = false keeps the assignment step's counters (the update only adds to
// `empty` and `error_flags`, which the caller has cleared).
// The incremental update is taken when the moved objects' entries are at most
// this share of all object entries (else the full reduction is cheaper).
constexpr int64_t kDeltaShare = 4;

ivf_status run_update(ivf_handle* h, const int32_t* assign, ivf_stats* stats,
                      bool clear = true) {
    const hipStream_t s = h->stream;
    const bool timed = stats && !h->fixed;
    if (timed) HIPCHK(h, hipEventRecord(h->ev[2], s));
    if (clear) HIPCHK(h, launch_clear_counters(h->cnt, s));
    const int o = h->cur, nb = 1 - h->cur;
    UpdateArgs a{};
    a.n = h->n; a.d = h->d; a.nnz = h->nnz; a.k = h->k;
    a.assign = assign;
    a.xt_obj = h->ov->xt_obj; a.xt_tv = h->ov->xt_tv;
    a.shift = h->ov->shift;
    a.keys = h->sc->keys; a.keys_alt = h->sc->keys_alt; a.pay = h->sc->pay;
    a.flag = h->sc->flag; a.segpos = h->sc->segpos; a.seg_acc = h->sc->seg_acc;
    a.seg_j = h->sc->seg_j; a.seg_t = h->sc->seg_t;
    a.size = h->size; a.cstart = h->cstart; a.nrm = h->nrm; a.objpart = h->objpart;
    a.newcnt = h->newcnt; a.scal = h->scal;
    a.norm_items = h->norm_items; a.norm_part = h->norm_part;
    a.old_ptr = h->mm_ptr[o]; a.old_idx = h->mm_idx[o]; a.old_val = h->mm_val[o];
    a.new_ptr = h->mm_ptr[nb];
    a.cnt = h->cnt;
    a.tmp = h->sc->tmp;
    // The sums table serves single handles outside graph capture whose member
    // sums are exact (no rounded term); it is valid again only once this
    // update has completed.
    const bool use_table = !h->fixed && h->owns_sc && !h->opt.full_update && h->ov->inexact == 0;
    const bool had_table = h->tab_valid;
    h->tab_valid = false;
    int64_t delta = -1;   // delta entries of the incremental update; -1: full reduction
    if (use_table && had_table) {
        HIPCHK(h, h->sc->ensure(0, 0, h->n + 1, s));
        if (!h->delta_off) HIPCHK(h, dalloc(&h->delta_off, h->n + 1));
        HIPCHK(h, launch_delta_count(h->ov->x_ptr, h->n, assign, h->tab_assign, h->k,
                                     h->delta_off, h->sc->tmp, s));
        int64_t e = 0;
        HIPCHK(h, hipMemcpyAsync(&e, h->delta_off + h->n, sizeof(int64_t), hipMemcpyDeviceToHost,
                                 s));
        HIPCHK(h, hipStreamSynchronize(s));
        if (e >= 0 && e <= h->nnz / kDeltaShare) delta = e;
    }
    if (delta >= 0) {
        const int nt = 1 - h->tc;
        ivf_status st = ensure_tab(h, nt, h->tab_n + delta);
        if (st != IVF_OK) return st;
        DeltaArgs da{};
        da.x_ptr = h->ov->x_ptr; da.x_idx = h->ov->x_idx; da.x_val = h->ov->x_val;
        da.n = h->n; da.d = h->d; da.k = h->k;
        da.assign = assign; da.old_assign = h->tab_assign;
        da.off = h->delta_off; da.entries = delta;
        da.shift = h->ov->shift; da.size = h->size; da.scal = h->scal;
        da.keys = h->sc->keys; da.keys_alt = h->sc->keys_alt;
        da.pay = h->sc->pay; da.pay_alt = reinterpret_cast<uint2*>(h->sc->seg_acc);
        da.flag = h->sc->flag; da.segpos = h->sc->segpos;
        da.dacc = h->sc->seg_acc; da.dj = h->sc->seg_j; da.dt = h->sc->seg_t;
        da.ins = h->sc->vals; da.ins_lb = h->sc->vals_alt; da.ipos = h->sc->keys_alt;
        da.tab_n = h->tab_n; da.cstart = h->cstart;
        da.tab_j = h->tab_j[h->tc]; da.tab_t = h->tab_t[h->tc]; da.tab_acc = h->tab_acc[h->tc];
        da.add = h->merge_add; da.cs = h->merge_cs;
        da.new_j = h->tab_j[nt]; da.new_t = h->tab_t[nt]; da.new_acc = h->tab_acc[nt];
        da.tmp = h->sc->tmp;
        HIPCHK(h, launch_delta_update(da, s));
        a.seg_acc = h->tab_acc[nt]; a.seg_j = h->tab_j[nt]; a.seg_t = h->tab_t[nt];
        HIPCHK(h, launch_update_norms(a, s));
    } else {
        HIPCHK(h, launch_update_sums(a, s));
    }
    int64_t nnz_new = 0, segs = 0;
    if (!h->fixed) {
        HIPCHK(h, hipMemcpyAsync(&nnz_new, h->mm_ptr[nb] + h->k, sizeof(int64_t),
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipMemcpyAsync(&segs, h->scal + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        ivf_status st = ensure_mm(h, nb, nnz_new);
        if (st != IVF_OK) return st;
    }
    a.new_cap = h->mm_cap[nb];
    a.new_idx = h->mm_idx[nb];
    a.new_val = h->mm_val[nb];
    a.new_row = h->mm_row[nb];
    HIPCHK(h, launch_update_fill(a, s));
    HIPCHK(h, launch_objective_exact(h->objpart, h->k, h->dscal + 1, s));
    // the table of this update's sums, for the next one
    if (delta >= 0) {
        h->tc = 1 - h->tc;
        h->tab_n = segs;
    } else if (use_table) {
        ivf_status st = ensure_tab(h, h->tc, segs);
        if (st != IVF_OK) return st;
        HIPCHK(h, launch_copy_table(h->sc->seg_j, h->sc->seg_t, h->sc->seg_acc, h->scal, segs,
                                    h->tab_j[h->tc], h->tab_t[h->tc], h->tab_acc[h->tc], s));
        h->tab_n = segs;
    }
    if (use_table) {
        if (!h->tab_assign) HIPCHK(h, dalloc(&h->tab_assign, std::max<int64_t>(h->n, 1)));
        HIPCHK(h, hipMemcpyAsync(h->tab_assign, assign, (size_t)h->n * sizeof(int32_t),
                                 hipMemcpyDeviceToDevice, s));
    }
    ivf_status st = rebuild_ivf(h, nb, nnz_new, h->fixed ? h->mm_ptr[nb] + h->k : nullptr);
    if (st != IVF_OK) return st;
    h->tab_valid = use_table;
    h->cur = nb;
    h->nnzM = nnz_new;
    h->nnzM_known = !h->fixed;
    h->has_means = true;
    if (timed) {
        HIPCHK(h, hipEventRecord(h->ev[3], s));
        HIPCHK(h, hipStreamSynchronize(s));
        Counters c;
        double ds[2];
        HIPCHK(h, hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
        HIPCHK(h, hipMemcpy(ds, h->dscal, sizeof(ds), hipMemcpyDeviceToHost));
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
        stats->objective_exact = ds[1];
        stats->empty_clusters = (int64_t)c.empty;
        stats->nnz_means = nnz_new;
        stats->inexact_terms = h->ov->inexact;
        stats->update_ms = ms;
        stats->update_delta_entries = delta;
    }
    return IVF_OK;
}

WalkArgs walk_args(ivf_handle* h) {
    const Plan& p = h->plan;
    WalkArgs w{};
    w.x_ptr = h->ov->x_ptr; w.x_idx = h->ov->x_idx; w.x_val = h->ov->x_val; w.n = h->n;
    w.desc = h->desc; w.post = h->post; w.slab = h->slab;
    w.k = h->k; w.k_r = p.k_r; w.R = p.R; w.chunk = p.chunk; w.tile_stride = p.tile_stride;
    w.items_per_range = (h->n + p.chunk - 1) / p.chunk;
    w.cnt = h->cnt; w.rec = h->rec;
    return w;
}

// Per-call scratch of an assignment step: the previous assignment, the walk's
// range records [n * R] and the FP64 re-score queue [n].  The handle's own
// buffers, or (ivf_assign_static) the library's fixed per-device array.
struct AssignBufs {
    int32_t* prev;
    RangeRec* rec;
    int32_t* rescore_list;
};

AssignBufs handle_bufs(ivf_handle* h) { return AssignBufs{h->prev, h->rec, h->rescore_list}; }

// Assignment step after the walk: merge, FP64 re-score, objective.  R: the
// range records per object (0: the plan's cluster ranges).
// R, rec, fixed_scale: records of another walk (IVFD's, R per object, of
// fixed-point sums at that scale); 0 / null: the plan's cluster ranges.
// bufs: the step's per-call scratch (null: the handle's buffers).
ivf_status assign_finish(ivf_handle* h, int32_t* assign, int32_t R = 0,
                         const RangeRec* rec = nullptr, double fixed_scale = 0.0,
                         const AssignBufs* bufs = nullptr) {
    const hipStream_t s = h->stream;
    const Plan& p = h->plan;
    const AssignBufs b = bufs ? *bufs : handle_bufs(h);
    MergeArgs m{};
    m.x_ptr = h->ov->x_ptr; m.n = h->n; m.R = R > 0 ? R : p.R;
    m.valtype = h->opt.valtype; m.certify = h->opt.certify; m.force_rescore = h->opt.force_rescore;
    m.fixed_scale = fixed_scale;
    m.vmax = h->ov->vmax;
    m.rec = rec ? rec : b.rec; m.prev = b.prev; m.assign = assign; m.rho = h->rho;
    m.best = h->best; m.best_id = h->best_id; m.second = h->second; m.flags = h->flags;
    m.rescore_list = b.rescore_list; m.cnt = h->cnt;
    HIPCHK(h, launch_merge(m, s));
    if (h->opt.certify) {
        RescoreArgs r{};
        r.w = walk_args(h);
        r.w.rec = b.rec;
        r.mm_ptr = h->mm_ptr[h->cur]; r.mm_idx = h->mm_idx[h->cur]; r.mm_val = h->mm_val[h->cur];
        r.valtype = h->opt.valtype;
        r.fixed_scale = fixed_scale;
        r.vmax = h->ov->vmax;
        r.rec = rec ? nullptr : b.rec;   // another walk's records bound other ranges
        r.rescore_list = b.rescore_list; r.prev = b.prev; r.assign = assign; r.rho = h->rho;
        r.best = h->best; r.best_id = h->best_id; r.cnt = h->cnt;
        HIPCHK(h, launch_rescore(r, h->rescore_waves, h->rescore_grid, s));
    }
    HIPCHK(h, launch_objective(h->rho, assign, b.prev, h->n, h->part, kObjBlocks, h->dscal,
                               h->cnt, s));
    return IVF_OK;
}

ivf_status assign_stats(ivf_handle* h, ivf_stats* stats, bool timed) {
    Counters c;
    double obj = 0.0;
    HIPCHK(h, hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(&obj, h->dscal, sizeof(obj), hipMemcpyDeviceToHost));
    float ms = 0.f, wms = 0.f;
    if (timed) {
        HIPCHK(h, hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
        HIPCHK(h, hipEventElapsedTime(&wms, h->ev[4], h->ev[5]));
    }
    double bound, err;
    std::memcpy(&bound, &c.max_bound_bits, sizeof(double));
    std::memcpy(&err, &c.max_err_bits, sizeof(double));
    stats->objective = obj;
    stats->objective_bound = bound;
    stats->changed = (int64_t)c.changed;
    stats->certified = (int64_t)c.certified;
    stats->rescored = (int64_t)c.n_rescore;
    stats->zero_overlap = (int64_t)c.zero_overlap;
    stats->mult_adds = (int64_t)c.mult;
    stats->max_rel_err_rescored = err;
    stats->assign_ms = ms;
    stats->walk_ms = wms;
    stats->objective_exact = std::nan("");
    stats->empty_clusters = -1;
    stats->nnz_means = h->nnzM_known ? h->nnzM : -1;
    stats->inexact_terms = h->ov->inexact;
    stats->update_ms = 0.f;
    stats->update_delta_entries = -1;
    return IVF_OK;
}

// The objects' inverted file for IVFD with n_r objects per range, built
// once per object set (and again if n_r changes).
ivf_status ensure_object_ivf(ivf_handle* h, int32_t n_r) {
    ObjView* ov = h->ov;
    if (ov->o_nr == n_r) return IVF_OK;
    dfree(ov->optr);
    dfree(ov->opost);
    ov->o_nr = 0;
    const int64_t R = (h->n + n_r - 1) / n_r;
    const int64_t nkeys = R * h->d;
    if (nkeys + 1 >= ((int64_t)1 << 32))
        return fail(h, IVF_ERR_CAPACITY, "IVFD: ranges x terms >= 2^32; use larger ranges");
    ivf_status st = ensure_scratch(h, std::max<int64_t>(h->nnz, 1));
    if (st != IVF_OK) return st;
    HIPCHK(h, dalloc(&ov->optr, nkeys + 1));
    HIPCHK(h, dalloc(&ov->opost, h->nnz));
    int32_t* rowid = nullptr;
    HIPCHK(h, dalloc(&rowid, h->nnz));
    Scratch* sc = h->sc;
    hipError_t e = launch_row_ids(ov->x_ptr, h->n, rowid, h->stream);
    if (e == hipSuccess)
        e = launch_ivfd_build(rowid, ov->x_idx, ov->x_val, h->nnz, n_r, h->d, nkeys, sc->keys,
                              sc->vals, sc->keys_alt, sc->vals_alt, sc->iota, sc->tmp, ov->optr,
                              ov->opost, h->stream);
    if (e == hipSuccess) e = launch_clear_counters(h->cnt, h->stream);
    if (e == hipSuccess)
        e = launch_max_row_norm(ov->x_ptr, ov->x_val, nullptr, h->n, &h->cnt->norm_bits, h->stream);
    Counters c;
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost);
    dfree(rowid);
    if (e != hipSuccess)
        return fail(h, IVF_ERR_HIP, std::string("IVFD build: ") + hipGetErrorString(e));
    std::memcpy(&ov->o_maxnorm, &c.norm_bits, sizeof(double));
    ov->o_nr = n_r;
    ov->o_R = R;
    return IVF_OK;
}

int occupancy_grid(int cus, const void* kernel, int waves, int lds) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave * waves,
                                                     (size_t)lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

// Launch shape of the FP64 re-score: as many waves per workgroup (each with
// its own tile) as fit the LDS, up to 8, and a persistent grid.
void plan_rescore(ivf_handle* h) {
    const int tile_bytes = h->plan.tile_stride * 4;
    h->rescore_waves = std::max(1, std::min(8, kLdsBytes / std::max(tile_bytes, 1)));
    h->rescore_grid = occupancy_grid(h->cus, rescore_kernel_ptr(h->opt.valtype), h->rescore_waves,
                                     h->rescore_waves * tile_bytes);
}

// Validation, term-major view and fixed-point scales of one object set.
ivf_status build_objview(ivf_handle* h, const ivf_csr* X) {
    ObjView* ov = h->ov;
    ov->x_ptr = X->indptr; ov->x_idx = X->indices; ov->x_val = X->values;
    ov->n = X->n; ov->d = X->d; ov->nnz = X->nnz;
    const int64_t n = X->n, d = X->d, nnz = X->nnz;
    HIPCHK(h, launch_clear_counters(h->cnt, h->stream));
    ObjectView xv{X->indptr, X->indices, X->values, n, d, nnz};
    HIPCHK(h, launch_validate_objects(xv, h->cnt, h->stream));
    Counters vc;
    ivf_status st = read_errors(h, "objects", &vc);
    if (st != IVF_OK) return st;
    std::memcpy(&ov->vmax, &vc.vmax_bits, sizeof(double));
    ov->nmax = (int64_t)vc.nmax;
    st = ensure_scratch(h, std::max<int64_t>(nnz, 1));
    if (st != IVF_OK) return st;
    Scratch* sc = h->sc;
    int32_t* rowid = nullptr;
    HIPCHK(h, dalloc(&rowid, nnz));
    HIPCHK(h, dalloc(&ov->xt_obj, nnz));
    HIPCHK(h, dalloc(&ov->xt_tv, nnz));
    if (nnz > 0) {
        // stable sort of (term, position): positions ascend with objects
        HIPCHK(h, launch_row_ids(X->indptr, n, rowid, h->stream));
        HIPCHK(h, launch_copy_keys(X->indices, sc->keys, nnz, h->stream));
        int bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) <= d - 1) ++bits;
        HIPCHK(h, radix_sort_pairs(sc->keys, sc->vals, sc->keys_alt, sc->vals_alt, nnz, bits,
                                   sc->tmp, h->stream, sc->iota));
        HIPCHK(h, launch_build_xt(sc->keys, sc->vals, rowid, X->values, nnz, ov->xt_obj,
                                  ov->xt_tv, h->stream));
    }
    int32_t *emin = nullptr, *emax = nullptr, *tcount = nullptr;
    HIPCHK(h, dalloc(&emin, d));
    HIPCHK(h, dalloc(&emax, d));
    HIPCHK(h, dalloc(&tcount, d));
    HIPCHK(h, dalloc(&ov->shift, d));
    HIPCHK(h, launch_term_shift(X->indices, X->values, nnz, d, emin, emax, tcount, ov->shift,
                                h->cnt, h->stream));
    Counters c;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
    ov->inexact = (int64_t)c.inexact;
    (void)hipFree(rowid);
    (void)hipFree(emin);
    (void)hipFree(emax);
    (void)hipFree(tcount);
    return IVF_OK;
}

// Plan-dependent buffers (one range record per object and range, one slice
// descriptor per term and range).
ivf_status alloc_plan_buffers(ivf_handle* h) {
    dfree(h->desc);
    dfree(h->dsz);
    dfree(h->rec);
    HIPCHK(h, dalloc(&h->desc, h->d * (int64_t)h->plan.R));
    HIPCHK(h, dalloc(&h->dsz, h->d * (int64_t)h->plan.R + 1));
    HIPCHK(h, dalloc(&h->rec, h->n * (int64_t)h->plan.R));
    return IVF_OK;
}

// Everything a handle owns besides the shared view and scratch.
ivf_status alloc_handle(ivf_handle* h) {
    const int64_t n = h->n, d = h->d;
    const int32_t k = h->k;
    HIPCHK(h, dalloc(&h->size, k));
    HIPCHK(h, dalloc(&h->cstart, (int64_t)k + 1));
    HIPCHK(h, dalloc(&h->newcnt, (int64_t)k + 1));
    HIPCHK(h, dalloc(&h->scal, 4));
    HIPCHK(h, dalloc(&h->nrm, k));
    HIPCHK(h, dalloc(&h->objpart, k));
    HIPCHK(h, dalloc(&h->norm_items, (int64_t)k + 1));
    HIPCHK(h, dalloc(&h->norm_part, 2 * norm_item_bound(k, h->nnz)));
    for (int b = 0; b < 2; ++b) {
        HIPCHK(h, dalloc(&h->mm_ptr[b], (int64_t)k + 1));
        HIPCHK(h, hipMemsetAsync(h->mm_ptr[b], 0, sizeof(int64_t) * ((size_t)k + 1), h->stream));
    }
    ivf_status st = ensure_mm(h, 0, 1);
    if (st != IVF_OK) return st;
    st = ensure_mm(h, 1, 1);
    if (st != IVF_OK) return st;
    HIPCHK(h, dalloc(&h->ivf_ptr, d + 1));
    st = alloc_plan_buffers(h);
    if (st != IVF_OK) return st;
    st = ensure_ivf(h, 1);
    if (st != IVF_OK) return st;
    HIPCHK(h, dalloc(&h->prev, n));
    HIPCHK(h, dalloc(&h->seed_assign, n));
    HIPCHK(h, dalloc(&h->rho, n));
    HIPCHK(h, dalloc(&h->best, n));
    HIPCHK(h, dalloc(&h->second, n));
    HIPCHK(h, dalloc(&h->best_id, n));
    HIPCHK(h, dalloc(&h->flags, n));
    HIPCHK(h, dalloc(&h->rescore_list, n));
    HIPCHK(h, dalloc(&h->part, kObjBlocks));
    HIPCHK(h, dalloc(&h->dscal, 4));
    HIPCHK(h, walk_set_lds_limit(kLdsBytes));
    h->walk_grid = occupancy_grid(h->cus, walk_kernel_ptr(h->opt.valtype, h->plan.k_r),
                                  h->plan.waves, h->plan.lds_bytes);
    plan_rescore(h);
    return IVF_OK;
}

ivf_status check_csr(const ivf_csr* X, int32_t k) {
    if (!X) return fail(nullptr, IVF_ERR_ARG, "null argument");
    if (X->n < 1 || X->d < 1 || X->nnz < 0) return fail(nullptr, IVF_ERR_ARG, "bad sizes");
    if (!X->indptr || (X->nnz > 0 && (!X->indices || !X->values)))
        return fail(nullptr, IVF_ERR_ARG, "null object arrays");
    if (k < 1 || (int64_t)k > X->n) return fail(nullptr, IVF_ERR_ARG, "k outside [1, n]");
    if (k >= (1 << 24)) return fail(nullptr, IVF_ERR_CAPACITY, "k >= 2^24");
    if (X->nnz >= ((int64_t)1 << 31) - 1 || X->n >= ((int64_t)1 << 31) - 1 ||
        X->d >= ((int64_t)1 << 31) - 1)
        return fail(nullptr, IVF_ERR_CAPACITY, "n, d or nnz >= 2^31");
    return IVF_OK;
}

// A handle on X with k clusters.  sc / ov: shared scratch and view, or null
// to create owned ones.
ivf_status create_handle(const ivf_csr* X, int32_t k, const ivf_options& o, Scratch* sc,
                         ObjView* ov, ivf_handle** out) {
    *out = nullptr;
    Plan plan;
    std::string perr;
    ivf_status pst = make_plan(k, &o, &plan, &perr);
    if (pst != IVF_OK) return fail(nullptr, pst, perr);
    ivf_handle* h = new (std::nothrow) ivf_handle();
    if (!h) return fail(nullptr, IVF_ERR_OOM, "host allocation failed");
    h->n = X->n; h->d = X->d; h->nnz = X->nnz; h->k = k;
    h->opt = o;
    h->stream = reinterpret_cast<hipStream_t>(o.stream);
    h->plan = plan;
    h->sc = sc ? sc : new (std::nothrow) Scratch();
    h->owns_sc = !sc;
    h->ov = ov ? ov : new (std::nothrow) ObjView();
    h->owns_ov = !ov;
    auto bail = [&](ivf_status st) {
        g_build_error = h->err;
        free_handle(h);
        delete h;
        return st;
    };
    if (!h->sc || !h->ov) return bail(fail(h, IVF_ERR_OOM, "host allocation failed"));
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device);
    for (auto& ev : h->ev)
        if (e == hipSuccess) e = hipEventCreate(&ev);
    if (e == hipSuccess) e = dalloc(&h->cnt, 1);
    if (e == hipSuccess) e = launch_clear_counters(h->cnt, h->stream);
    if (e != hipSuccess)
        return bail(fail(h, e == hipErrorOutOfMemory ? IVF_ERR_OOM : IVF_ERR_HIP,
                         std::string("device setup: ") + hipGetErrorString(e)));
    ivf_status st = IVF_OK;
    if (!ov) st = build_objview(h, X);
    else st = ensure_scratch(h, std::max<int64_t>(X->nnz, 1));
    // means of the update are unit-norm: the objects alone must keep scores finite
    if (st == IVF_OK) st = check_value_range(h, 1.0);
    if (st == IVF_OK) st = alloc_handle(h);
    if (st == IVF_OK) {
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) st = fail(h, IVF_ERR_HIP, hipGetErrorString(e));
    }
    if (st != IVF_OK) return bail(st);
    *out = h;
    return IVF_OK;
}

}  // namespace


// ------------------------------------------------------------------ batches
struct ivf_batch {
    std::vector<ivf_handle*> h;
    std::vector<ObjView*> views;
    // After the walk, the instances' merges and updates run on kLanes streams,
    // forked from and joined back into the batch stream; small instances
    // leave most of the GPU idle on their own.  Instances go to lanes largest
    // first, each to the lane with the fewest object nonzeros so far.  Each
    // lane has its own sort/segment scratch, sized for its largest instance:
    // instances of one lane run one after another.
    static constexpr int kLanes = 4;
    Scratch* lane_sc[kLanes] = {};
    hipStream_t lane[kLanes] = {};
    std::vector<int> lane_of;   // per instance
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kLanes] = {};
    ivf_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cus = 0;
    int32_t kr_max = 0, waves = 0, tile_stride = 0, grid = 0;
    bool tuned = false;
    WalkArgs* d_args = nullptr;
    int64_t* d_item_off = nullptr;
    Counters** d_cnt = nullptr;                // every instance's counters
    unsigned long long* d_flags = nullptr;     // their error flags, gathered
    // two recorded iterations: every instance's means move from its current
    // buffer to the other in exec[0] and back in exec[1]; phase: the next one
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int phase = 0;
    std::vector<int32_t*> captured_assign;
    int eager_left = 2;      // eager iterations that size the fixed capacities
    double slack_frac = 0.5;  // fixed capacity = need * (1 + slack_frac) + slack_abs
    int64_t slack_abs = 1024;
    int32_t recoveries = 0;   // replays whose new means overflowed a fixed capacity
    int32_t captures = 0;     // times the iteration was recorded
    std::vector<float> tune_ms;   // autotuner: walk time of each candidate tried
    std::vector<int32_t> tune_shape;   // and its (clusters per tile, waves) pairs
    std::vector<float> tune_theta;     // dense-slab thresholds tried on the chosen shape
    std::vector<float> tune_theta_ms;  // and the walk time with each
    hipEvent_t ev[2] = {nullptr, nullptr};
    // device real-time clock read just before and just after the batched walk:
    // kernel nodes, so graph replays time the walk too
    unsigned long long* d_stamp = nullptr;
    unsigned long long* d_work = nullptr;   // work-item counter of the batched walk
    int clock_khz = 0;
    std::string err;
};

// ------------------------------------------------ allocation-free assignment
// One fixed array per GPU for ivf_assign_static: the per-call scratch of an
// assignment step (previous assignment, FP64 re-score queue, range records),
// each part starting on a 256-byte boundary.  In host code `scratch` names a
// host-side stand-in; the device address comes from hipGetSymbolAddress, once
// per device, and only that address is handed to kernels and copies.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

ivf_status bfail(ivf_batch* b, ivf_status st, const std::string& msg) {
    if (b) b->err = msg;
    else g_build_error = msg;
    return st;
}

#define BHIP(b, call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return bfail((b), e_ == hipErrorOutOfMemory ? IVF_ERR_OOM : IVF_ERR_HIP,     \
                         std::string(#call) + ": " + hipGetErrorString(e_));             \
    } while (0)

__global__ void k_stamp(unsigned long long* out) {
    if (threadIdx.x == 0) *out = wall_clock64();
}

void drop_graphs(ivf_batch* b) {
    for (auto& e : b->exec)
        if (e) { (void)hipGraphExecDestroy(e); e = nullptr; }
}

ivf_status upload_args(ivf_batch* b) {
    const int32_t count = (int32_t)b->h.size();
    std::vector<WalkArgs> args(count);
    std::vector<int64_t> off(count + 1, 0);
    for (int32_t i = 0; i < count; ++i) {
        args[i] = walk_args(b->h[i]);
        off[i + 1] = off[i] + args[i].items_per_range * args[i].R;
    }
    BHIP(b, hipMemcpyAsync(b->d_args, args.data(), sizeof(WalkArgs) * count,
                           hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_item_off, off.data(), sizeof(int64_t) * (count + 1),
                           hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return IVF_OK;
}

// Re-plan every instance for (kr_max, waves); with means present, their
// inverted files are rebuilt for the new ranges.
ivf_status batch_plan(ivf_batch* b, int32_t kr_max, int32_t waves) {
    ivf_options o = b->opt;
    o.cluster_range = kr_max;
    o.waves_per_wg = 1;   // per-instance tiles are unused by the batched walk
    int32_t stride = 4;
    std::vector<Plan> plans;
    for (ivf_handle* h : b->h) {
        Plan p;
        std::string perr;
        ivf_status st = make_plan(h->k, &o, &p, &perr);
        if (st != IVF_OK) return bfail(b, st, perr);
        stride = std::max(stride, p.tile_stride);
        plans.push_back(p);
    }
    if ((int64_t)waves * stride * 4 > kLdsBytes) return bfail(b, IVF_ERR_ARG, "tiles exceed LDS");
    for (size_t i = 0; i < b->h.size(); ++i) {
        ivf_handle* h = b->h[i];
        const bool new_ranges = plans[i].R != h->plan.R;
        h->plan = plans[i];
        plan_rescore(h);
        if (new_ranges) {
            ivf_status st = alloc_plan_buffers(h);
            if (st != IVF_OK) return bfail(b, st, h->err);
        }
        ivf_status st = ensure_scratch(h, std::max<int64_t>(h->nnz, 1));
        if (st != IVF_OK) return bfail(b, st, h->err);
        if (h->has_means) {
            if (!h->nnzM_known) {
                BHIP(b, hipStreamSynchronize(b->stream));
                BHIP(b, hipMemcpy(&h->nnzM, h->mm_ptr[h->cur] + h->k, sizeof(int64_t),
                                  hipMemcpyDeviceToHost));
                h->nnzM_known = true;
            }
            st = rebuild_ivf(h, h->cur, h->nnzM, nullptr);
            if (st != IVF_OK) return bfail(b, st, h->err);
        }
    }
    b->kr_max = kr_max;
    b->waves = waves;
    b->tile_stride = stride;
    b->grid = occupancy_grid(b->cus, walk_batch_kernel_ptr(b->opt.valtype, stride), waves,
                             waves * stride * 4);
    drop_graphs(b);
    return upload_args(b);
}

// Device time of one batched walk on the current plan and means.
ivf_status time_batch_walk(ivf_batch* b, float* ms) {
    BHIP(b, hipEventRecord(b->ev[0], b->stream));
    BHIP(b, launch_walk_batch(b->d_args, b->d_item_off, (int32_t)b->h.size(), b->tile_stride,
                              b->opt.valtype, b->waves, b->grid, b->d_work, b->stream));
    BHIP(b, hipEventRecord(b->ev[1], b->stream));
    BHIP(b, hipEventSynchronize(b->ev[1]));
    BHIP(b, hipEventElapsedTime(ms, b->ev[0], b->ev[1]));
    return IVF_OK;
}

// Autotuner: time the batched walk on the current means for every candidate
// (clusters per tile, waves per workgroup) and keep the fastest; then, unless
// the caller fixed it, the dense-slab threshold on that shape.
ivf_status batch_autotune(ivf_batch* b) {
    // 640-wide tiles measured slowest on every mix tried; wider tiles favour
    // batches whose k spread past one 1280-wide range, 1024 the FP32 walk of
    // large k (the single-instance planner's choice)
    static const int32_t cand[][2] = {{1024, 8}, {1280, 8}, {2560, 4}, {2560, 8}, {5120, 4}};
    float best = 1e30f;
    int bi = 0;
    b->tune_ms.clear();
    b->tune_shape.clear();
    b->tune_theta.clear();
    b->tune_theta_ms.clear();
    for (int c = 0; c < (int)(sizeof(cand) / sizeof(cand[0])); ++c) {
        ivf_status st = batch_plan(b, cand[c][0], cand[c][1]);
        if (st != IVF_OK) return st;
        float ms = 0.f;
        st = time_batch_walk(b, &ms);
        if (st != IVF_OK) return st;
        b->tune_ms.push_back(ms);
        b->tune_shape.push_back(cand[c][0]);
        b->tune_shape.push_back(cand[c][1]);
        if (ms < best) { best = ms; bi = c; }
    }
    b->tuned = true;
    if (b->opt.dense_threshold > 0.f) return batch_plan(b, cand[bi][0], cand[bi][1]);
    // A higher threshold stores fewer, fuller slabs: fewer zero bytes read,
    // more (id, value) entries.  Mixes of many small instances measured
    // fastest above the default chosen for one large instance.  The shapes
    // were timed at each instance's default (dense_default); the thresholds
    // are then timed on the chosen shape, each for every instance.
    static const float thetas[] = {0.35f, 0.45f, 0.5f, 0.65f};
    float t_best = thetas[0];
    best = 3.4e38f;
    for (float t : thetas) {
        for (ivf_handle* h : b->h) h->opt.dense_threshold = t;
        ivf_status st = batch_plan(b, cand[bi][0], cand[bi][1]);
        if (st != IVF_OK) return st;
        float ms = 0.f;
        st = time_batch_walk(b, &ms);
        if (st != IVF_OK) return st;
        b->tune_theta.push_back(t);
        b->tune_theta_ms.push_back(ms);
        if (ms < best) { best = ms; t_best = t; }
    }
    for (ivf_handle* h : b->h) h->opt.dense_threshold = t_best;
    return batch_plan(b, cand[bi][0], cand[bi][1]);
}

// One Lloyd iteration of every instance.  Eager (synchronises, may grow
// buffers) or, with every handle fixed, recordable in a graph.
ivf_status batch_iteration(ivf_batch* b, int32_t* const* assign, bool eager) {
    const hipStream_t s = b->stream;
    const int32_t count = (int32_t)b->h.size();
    for (int32_t i = 0; i < count; ++i) {
        ivf_handle* h = b->h[i];
        HIPCHK(h, launch_clear_counters(h->cnt, s));
        HIPCHK(h, hipMemcpyAsync(h->prev, assign[i], sizeof(int32_t) * (size_t)h->n,
                                 hipMemcpyDeviceToDevice, s));
    }
    k_stamp<<<1, 64, 0, s>>>(b->d_stamp);
    BHIP(b, launch_walk_batch(b->d_args, b->d_item_off, count, b->tile_stride, b->opt.valtype,
                              b->waves, b->grid, b->d_work, s));
    k_stamp<<<1, 64, 0, s>>>(b->d_stamp + 1);
    BHIP(b, hipGetLastError());
    // merges and updates on the lanes: fork after the walk, join before returning
    BHIP(b, hipEventRecord(b->fork_ev, s));
    for (int l = 0; l < ivf_batch::kLanes; ++l) BHIP(b, hipStreamWaitEvent(b->lane[l], b->fork_ev, 0));
    ivf_status st = IVF_OK;
    int32_t failed = -1;
    for (int32_t i = 0; i < count && st == IVF_OK; ++i) {
        ivf_handle* h = b->h[i];
        h->stream = b->lane[b->lane_of[i]];
        st = assign_finish(h, assign[i]);
        if (st == IVF_OK) st = run_update(h, assign[i], nullptr, false);
        h->stream = s;
        if (st != IVF_OK) failed = i;
    }
    // the join is recorded on every path, so a capture always ends joined
    for (int l = 0; l < ivf_batch::kLanes; ++l) {
        BHIP(b, hipEventRecord(b->join_ev[l], b->lane[l]));
        BHIP(b, hipStreamWaitEvent(s, b->join_ev[l], 0));
    }
    if (st != IVF_OK) return bfail(b, st, b->h[failed]->err);
    if (eager) return upload_args(b);   // slab pointers may have moved
    return IVF_OK;
}

ivf_status batch_fix_capacities(ivf_batch* b) {
    // capacities: what the eager iterations needed plus the slack; slices that
    // would not fit a slab later stay sparse, means that would not fit are flagged
    BHIP(b, hipStreamSynchronize(b->stream));
    for (ivf_handle* h : b->h) {
        h->fixed = false;
        if (!h->nnzM_known) {   // after replays the count lives on the device
            BHIP(b, hipMemcpy(&h->nnzM, h->mm_ptr[h->cur] + h->k, sizeof(int64_t),
                              hipMemcpyDeviceToHost));
            h->nnzM_known = true;
        }
        const int64_t need = std::max<int64_t>(h->nnzM, 1);
        const int64_t cap = need + (int64_t)((double)need * b->slack_frac) + b->slack_abs;
        for (int m = 0; m < 2; ++m) {   // the current means are carried over
            ivf_status st = ensure_mm(h, m, cap, m == h->cur ? h->nnzM : 0);
            if (st != IVF_OK) return bfail(b, st, h->err);
        }
        ivf_status st = ensure_ivf(h, std::max(h->mm_cap[0], h->mm_cap[1]));
        if (st != IVF_OK) return bfail(b, st, h->err);
        st = ensure_slab(h, h->slab_need + (int64_t)((double)h->slab_need * b->slack_frac) +
                                b->slack_abs);
        if (st != IVF_OK) return bfail(b, st, h->err);
        // the inverted file and slabs may have been reallocated: rebuild them
        st = rebuild_ivf(h, h->cur, h->nnzM, nullptr);
        if (st != IVF_OK) return bfail(b, st, h->err);
    }
    for (ivf_handle* h : b->h) h->fixed = true;
    drop_graphs(b);
    return upload_args(b);
}

ivf_status batch_capture(ivf_batch* b, int32_t* const* assign) {
    drop_graphs(b);
    for (int g = 0; g < 2; ++g) {
        hipGraph_t graph = nullptr;
        BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        ivf_status st = batch_iteration(b, assign, false);
        hipError_t ee = hipStreamEndCapture(b->stream, &graph);
        if (st != IVF_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        BHIP(b, ee);
        hipError_t ei = hipGraphInstantiate(&b->exec[g], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        BHIP(b, ei);
    }
    // recording flipped every handle's buffer parity twice: back where it was
    b->captured_assign.assign(assign, assign + b->h.size());
    b->phase = 0;
    ++b->captures;
    return IVF_OK;
}

__global__ void k_gather_flags(Counters* const* cnts, int32_t count, unsigned long long* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = cnts[i]->error_flags;
}

// The assignment step with its per-call scratch in `b`.
ivf_status assign_with(ivf_handle* h, int32_t* assign, ivf_stats* stats, const AssignBufs& b) {
    const hipStream_t s = h->stream;
    const Plan& p = h->plan;
    if (stats) HIPCHK(h, hipEventRecord(h->ev[0], s));
    HIPCHK(h, launch_clear_counters(h->cnt, s));
    HIPCHK(h, hipMemcpyAsync(b.prev, assign, sizeof(int32_t) * (size_t)h->n,
                             hipMemcpyDeviceToDevice, s));
    WalkArgs w = walk_args(h);
    w.rec = b.rec;
    if (stats) HIPCHK(h, hipEventRecord(h->ev[4], s));
    HIPCHK(h, launch_walk(w, h->opt.valtype, p.waves, p.lds_bytes, h->walk_grid, s));
    if (stats) HIPCHK(h, hipEventRecord(h->ev[5], s));
    ivf_status st = assign_finish(h, assign, 0, nullptr, 0.0, &b);
    if (st != IVF_OK) return st;
    if (stats) {
        HIPCHK(h, hipEventRecord(h->ev[1], s));
        HIPCHK(h, hipStreamSynchronize(s));
        return assign_stats(h, stats, true);
    }
    return IVF_OK;
}

// ------------------------------------------------ allocation-free assignment
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t static_scratch_need(const ivf_handle* h) {
    const size_t n = (size_t)h->n;
    return align256(n * sizeof(int32_t)) * 2 + n * (size_t)h->plan.R * sizeof(RangeRec);
}

// The device address of this device's array, looked up on the first call on it.
ivf_status static_scratch(ivf_handle* h, int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(h, IVF_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                            hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return IVF_OK;
}

}  // namespace

// --------------------------------------------------------------------- C ABI
extern "C" {

void ivf_default_options(ivf_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->valtype = IVF_VAL_F32;
    o->certify = 1;
}

const char* ivf_status_str(int32_t s) {
    switch (s) {
        case IVF_OK: return "IVF_OK";
        case IVF_ERR_ARG: return "IVF_ERR_ARG";
        case IVF_ERR_UNSORTED: return "IVF_ERR_UNSORTED";
        case IVF_ERR_NONFINITE: return "IVF_ERR_NONFINITE";
        case IVF_ERR_NEGATIVE: return "IVF_ERR_NEGATIVE";
        case IVF_ERR_CAPACITY: return "IVF_ERR_CAPACITY";
        case IVF_ERR_OOM: return "IVF_ERR_OOM";
        case IVF_ERR_HIP: return "IVF_ERR_HIP";
        case IVF_ERR_STATE: return "IVF_ERR_STATE";
        default: return "IVF_UNKNOWN";
    }
}

const char* ivf_last_error(const ivf_handle* h) {
    return h ? h->err.c_str() : g_build_error.c_str();
}

ivf_status ivf_plan_shape(int32_t k, const ivf_options* opts, int32_t plan[7]) {
    if (!plan) return IVF_ERR_ARG;
    Plan p;
    ivf_status st = make_plan(k, opts, &p, &g_build_error);
    if (st != IVF_OK) return st;
    plan[0] = p.k_r; plan[1] = p.R; plan[2] = p.waves; plan[3] = p.chunk;
    plan[4] = p.k_r64; plan[5] = p.R64; plan[6] = p.lds_bytes;
    return IVF_OK;
}

ivf_status ivf_get_plan(const ivf_handle* h, int32_t plan[7]) {
    if (!h || !plan) return IVF_ERR_ARG;
    const Plan& p = h->plan;
    plan[0] = p.k_r; plan[1] = p.R; plan[2] = p.waves; plan[3] = p.chunk;
    plan[4] = p.k_r64; plan[5] = p.R64; plan[6] = p.lds_bytes;
    return IVF_OK;
}

ivf_status ivf_cert_bound(int32_t valtype, int64_t nt, double vmax, double c[3]) {
    if (!c || valtype < IVF_VAL_F32 || valtype > IVF_VAL_F16 || nt < 0 || !(vmax >= 0.0) ||
        !std::isfinite(vmax))
        return IVF_ERR_ARG;
    cert_consts(valtype, nt, vmax, &c[0], &c[1], &c[2]);
    return IVF_OK;
}

ivf_status ivf_cert_bound_fixed(int64_t nt, double scale, double vmax, double c[3]) {
    if (!c || nt < 0 || !(scale > 0.0) || !std::isfinite(scale) || !(vmax >= 0.0) ||
        !std::isfinite(vmax))
        return IVF_ERR_ARG;
    cert_consts_fixed(nt, scale, vmax, &c[0], &c[1], &c[2]);
    return IVF_OK;
}

ivf_status ivf_build(const ivf_csr* X, int32_t k, const ivf_options* opts, ivf_handle** out) {
    if (out) *out = nullptr;
    if (!out) return fail(nullptr, IVF_ERR_ARG, "null argument");
    ivf_status st = check_csr(X, k);
    if (st != IVF_OK) return st;
    ivf_options o;
    ivf_default_options(&o);
    if (opts) o = *opts;
    if (o.valtype < IVF_VAL_F32 || o.valtype > IVF_VAL_F16)
        return fail(nullptr, IVF_ERR_ARG, "unknown valtype");
    return create_handle(X, k, o, nullptr, nullptr, out);
}

void ivf_destroy(ivf_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    free_handle(h);
    delete h;
}

ivf_status ivf_set_means(ivf_handle* h, const ivf_means* M) {
    if (!h || !M) return fail(h, IVF_ERR_ARG, "null argument");
    if (M->k != h->k || M->d != h->d || M->nnz < 0)
        return fail(h, IVF_ERR_ARG, "means k/d do not match the handle");
    if (!M->indptr || (M->nnz > 0 && (!M->indices || !M->values)))
        return fail(h, IVF_ERR_ARG, "null mean arrays");
    if (M->nnz >= ((int64_t)1 << 31) - 1) return fail(h, IVF_ERR_CAPACITY, "nnz >= 2^31");
    if (h->fixed) return fail(h, IVF_ERR_STATE, "capacities are fixed");
    HIPCHK(h, launch_clear_counters(h->cnt, h->stream));
    HIPCHK(h, launch_validate_means(M->indptr, M->indices, M->values, h->k, h->d, M->nnz, h->cnt,
                                    h->stream));
    Counters vc;
    ivf_status st = read_errors(h, "means", &vc);
    if (st != IVF_OK) return st;
    double mmax = 0.0;
    std::memcpy(&mmax, &vc.vmax_bits, sizeof(double));
    // rows the update keeps (empty clusters) may hold earlier means' values
    mmax = std::max(mmax, 1.0);
    st = check_value_range(h, mmax);
    if (st != IVF_OK) return st;
    const int b = h->cur;
    st = ensure_mm(h, b, M->nnz);
    if (st != IVF_OK) return st;
    HIPCHK(h, hipMemcpyAsync(h->mm_ptr[b], M->indptr, sizeof(int64_t) * ((size_t)h->k + 1),
                             hipMemcpyDeviceToDevice, h->stream));
    if (M->nnz > 0) {
        HIPCHK(h, hipMemcpyAsync(h->mm_idx[b], M->indices, sizeof(int32_t) * (size_t)M->nnz,
                                 hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->mm_val[b], M->values, sizeof(double) * (size_t)M->nnz,
                                 hipMemcpyDeviceToDevice, h->stream));
    }
    HIPCHK(h, launch_mean_rows(h->mm_ptr[b], h->k, h->mm_row[b], h->stream));
    st = rebuild_ivf(h, b, M->nnz, nullptr);
    if (st != IVF_OK) return st;
    h->nnzM = M->nnz;
    h->nnzM_known = true;
    h->has_means = true;
    h->mmax = mmax;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return IVF_OK;
}

ivf_status ivf_init_seeds(ivf_handle* h, const int32_t* seeds) {
    if (!h || !seeds) return fail(h, IVF_ERR_ARG, "null argument");
    if (h->fixed) return fail(h, IVF_ERR_STATE, "capacities are fixed");
    // start from empty means so that the singleton update defines every mean
    HIPCHK(h, hipMemsetAsync(h->mm_ptr[h->cur], 0, sizeof(int64_t) * ((size_t)h->k + 1),
                             h->stream));
    HIPCHK(h, launch_seed_assign(seeds, h->k, h->n, h->seed_assign, h->stream));
    ivf_status st = run_update(h, h->seed_assign, nullptr);
    if (st != IVF_OK) return st;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return IVF_OK;
}

ivf_status ivf_assign(ivf_handle* h, int32_t* assign, ivf_stats* stats) {
    if (!h || !assign) return fail(h, IVF_ERR_ARG, "null argument");
    if (!h->has_means) return fail(h, IVF_ERR_STATE, "no means: call ivf_set_means or ivf_init_seeds");
    return assign_with(h, assign, stats, handle_bufs(h));
}

ivf_status ivf_assign_static(ivf_handle* h, int32_t* assign, ivf_stats* stats) {
    if (!h || !assign) return fail(h, IVF_ERR_ARG, "null argument");
    if (!h->has_means) return fail(h, IVF_ERR_STATE, "no means: call ivf_set_means or ivf_init_seeds");
    const size_t need = static_scratch_need(h);
    if (need > kStaticScratchBytes)
        return fail(h, IVF_ERR_CAPACITY,
                    "ivf_assign_static: the step needs " + std::to_string(need) +
                        " bytes of scratch (n * (16 * ranges + 8), rounded), beyond the fixed " +
                        std::to_string(kStaticScratchBytes) + " bytes; use ivf_assign");
    int dev = -1;
    HIPCHK(h, hipGetDevice(&dev));
    if (dev != h->device)
        return fail(h, IVF_ERR_STATE, "ivf_assign_static: the handle's device must be current");
    if (dev < 0 || dev >= kMaxDevices) return fail(h, IVF_ERR_CAPACITY, "device index too large");
    unsigned char* base = nullptr;
    ivf_status st = static_scratch(h, dev, &base);
    if (st != IVF_OK) return st;
    const size_t n4 = align256((size_t)h->n * sizeof(int32_t));
    AssignBufs b{};
    b.prev = reinterpret_cast<int32_t*>(base);
    b.rescore_list = reinterpret_cast<int32_t*>(base + n4);
    b.rec = reinterpret_cast<RangeRec*>(base + 2 * n4);
    return assign_with(h, assign, stats, b);
}

ivf_status ivf_update(ivf_handle* h, const int32_t* assign, ivf_stats* stats) {
    if (!h || !assign) return fail(h, IVF_ERR_ARG, "null argument");
    return run_update(h, assign, stats);
}

ivf_status ivf_iterate(ivf_handle* h, int32_t iters, int32_t* assign, ivf_stats* per_iter) {
    if (!h || !assign || iters < 0) return fail(h, IVF_ERR_ARG, "bad argument");
    for (int32_t r = 0; r < iters; ++r) {
        ivf_stats* st = per_iter ? per_iter + r : nullptr;
        ivf_status e = ivf_assign(h, assign, st);
        if (e != IVF_OK) return e;
        e = run_update(h, assign, st);
        if (e != IVF_OK) return e;
    }
    return IVF_OK;
}

ivf_status ivf_converge(ivf_handle* h, int32_t max_iters, int32_t* assign, ivf_stats* per_iter,
                        int32_t* iters_done) {
    if (!h || !assign || !iters_done || max_iters < 0)
        return fail(h, IVF_ERR_ARG, "bad argument");
    *iters_done = 0;
    for (int32_t r = 0; r < max_iters; ++r) {
        ivf_stats st{};
        ivf_status e = ivf_assign(h, assign, &st);
        if (e != IVF_OK) return e;
        *iters_done = r + 1;
        if (st.changed == 0) {
            // the partition is the previous one, so the update would return
            // the same means: converged, and the update is skipped
            st.objective_exact = std::nan("");
            st.empty_clusters = -1;
            st.nnz_means = h->nnzM_known ? h->nnzM : -1;
            st.update_ms = 0.f;
            if (per_iter) per_iter[r] = st;
            return IVF_OK;
        }
        e = run_update(h, assign, &st);
        if (e != IVF_OK) return e;
        if (per_iter) per_iter[r] = st;
    }
    return IVF_OK;
}

ivf_status ivf_assign_ivfd(ivf_handle* h, int32_t objects_per_range, int32_t* assign,
                           ivf_stats* stats) {
    if (!h || !assign) return fail(h, IVF_ERR_ARG, "null argument");
    if (!h->has_means) return fail(h, IVF_ERR_STATE, "no means: call ivf_set_means or ivf_init_seeds");
    if (h->opt.valtype != IVF_VAL_F32)
        return fail(h, IVF_ERR_ARG, "IVFD scores in FP32: build the handle with FP32 values");
    if (h->fixed) return fail(h, IVF_ERR_STATE, "capacities are fixed");
    const int32_t n_r = objects_per_range > 0 ? objects_per_range : 16384;
    if (n_r != 4096 && n_r != 8192 && n_r != 16384)
        return fail(h, IVF_ERR_ARG, "objects_per_range must be 4096, 8192 or 16384");
    ivf_status st = ensure_object_ivf(h, n_r);
    if (st != IVF_OK) return st;
    const hipStream_t s = h->stream;
    const int32_t R = (int32_t)h->ov->o_R;
    // blocks of means: about four workgroups per compute unit
    const int32_t B = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(h->k, (4 * (int64_t)h->cus + R - 1) / R));
    if (h->n * (int64_t)B > h->ivfd_rec_cap) {
        dfree(h->ivfd_rec);
        h->ivfd_rec_cap = 0;
        HIPCHK(h, dalloc(&h->ivfd_rec, h->n * (int64_t)B));
        h->ivfd_rec_cap = h->n * (int64_t)B;
    }
    // fixed-point scale: every score is at most |x| |mu|, so with
    // 2^F * max|x| * max|mu| <= 2^31 no sum (with its roundings) reaches 2^32
    HIPCHK(h, launch_clear_counters(h->cnt, s));
    HIPCHK(h, launch_max_row_norm(h->mm_ptr[h->cur], nullptr, h->mm_val[h->cur], h->k,
                                  &h->cnt->norm_bits, s));
    Counters cn;
    HIPCHK(h, hipStreamSynchronize(s));
    HIPCHK(h, hipMemcpy(&cn, h->cnt, sizeof(cn), hipMemcpyDeviceToHost));
    double mnorm = 0.0;
    std::memcpy(&mnorm, &cn.norm_bits, sizeof(double));
    const double bound = h->ov->o_maxnorm * mnorm * (1.0 + 0x1p-20);
    int F = 60;
    if (bound > 0.0) F = std::min(60, std::max(-60, 31 - (int)std::ceil(std::log2(bound))));
    if (stats) HIPCHK(h, hipEventRecord(h->ev[0], s));
    HIPCHK(h, launch_clear_counters(h->cnt, s));
    HIPCHK(h, hipMemcpyAsync(h->prev, assign, sizeof(int32_t) * (size_t)h->n,
                             hipMemcpyDeviceToDevice, s));
    IvfdArgs a{};
    a.optr = h->ov->optr; a.opost = h->ov->opost;
    a.mm_ptr = h->mm_ptr[h->cur]; a.mm_idx = h->mm_idx[h->cur]; a.mm_val = h->mm_val[h->cur];
    a.n = h->n; a.d = h->d; a.k = h->k; a.R = R; a.n_r = n_r; a.B = B;
    a.scale = std::ldexp(1.0f, F);
    a.inv_scale = std::ldexp(1.0f, -F);
    a.rec = h->ivfd_rec; a.walked = &h->cnt->walked;
    if (stats) HIPCHK(h, hipEventRecord(h->ev[4], s));
    HIPCHK(h, launch_ivfd_walk(a, s));
    if (stats) HIPCHK(h, hipEventRecord(h->ev[5], s));
    HIPCHK(h, launch_ivfd_overlap(h->ov->x_ptr, h->ov->x_idx, h->n, B, h->ivf_ptr, h->ivfd_rec, s));
    st = assign_finish(h, assign, B, h->ivfd_rec, std::ldexp(1.0, F));
    if (st != IVF_OK) return st;
    if (stats) {
        HIPCHK(h, hipEventRecord(h->ev[1], s));
        HIPCHK(h, hipStreamSynchronize(s));
        st = assign_stats(h, stats, true);
        if (st != IVF_OK) return st;
        Counters c;
        HIPCHK(h, hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
        stats->mult_adds = (int64_t)c.walked;   // counted by the walk itself
    }
    return IVF_OK;
}

ivf_status ivf_get_means(ivf_handle* h, ivf_means* out) {
    if (!h || !out) return fail(h, IVF_ERR_ARG, "null argument");
    if (!h->has_means) return fail(h, IVF_ERR_STATE, "no means yet");
    const int b = h->cur;
    if (!h->nnzM_known) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        HIPCHK(h, hipMemcpy(&h->nnzM, h->mm_ptr[b] + h->k, sizeof(int64_t),
                            hipMemcpyDeviceToHost));
        h->nnzM_known = true;
    }
    out->k = h->k;
    out->d = h->d;
    if (!out->indptr) {
        out->nnz = h->nnzM;
        return IVF_OK;
    }
    if (out->nnz < h->nnzM || (h->nnzM > 0 && (!out->indices || !out->values)))
        return fail(h, IVF_ERR_ARG, "output buffers smaller than nnz");
    HIPCHK(h, hipMemcpyAsync(out->indptr, h->mm_ptr[b], sizeof(int64_t) * ((size_t)h->k + 1),
                             hipMemcpyDeviceToDevice, h->stream));
    if (h->nnzM > 0) {
        HIPCHK(h, hipMemcpyAsync(out->indices, h->mm_idx[b], sizeof(int32_t) * (size_t)h->nnzM,
                                 hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(out->values, h->mm_val[b], sizeof(double) * (size_t)h->nnzM,
                                 hipMemcpyDeviceToDevice, h->stream));
    }
    out->nnz = h->nnzM;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return IVF_OK;
}

ivf_status ivf_get_scores(ivf_handle* h, float* best, int32_t* best_id, float* second,
                          double* rho, uint8_t* flags) {
    if (!h) return IVF_ERR_ARG;
    const size_t n = (size_t)h->n;
    if (best) HIPCHK(h, hipMemcpyAsync(best, h->best, n * 4, hipMemcpyDeviceToDevice, h->stream));
    if (best_id)
        HIPCHK(h, hipMemcpyAsync(best_id, h->best_id, n * 4, hipMemcpyDeviceToDevice, h->stream));
    if (second)
        HIPCHK(h, hipMemcpyAsync(second, h->second, n * 4, hipMemcpyDeviceToDevice, h->stream));
    if (rho) HIPCHK(h, hipMemcpyAsync(rho, h->rho, n * 8, hipMemcpyDeviceToDevice, h->stream));
    if (flags) HIPCHK(h, hipMemcpyAsync(flags, h->flags, n, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return IVF_OK;
}

// ------------------------------------------------------------------ batches
void ivf_batch_destroy(ivf_batch* b);

ivf_status ivf_batch_build(int32_t count, const ivf_csr* X, const int32_t* k,
                           const ivf_options* opts, ivf_batch** out) {
    if (out) *out = nullptr;
    if (!out || !X || !k || count < 1) return bfail(nullptr, IVF_ERR_ARG, "bad argument");
    for (int32_t i = 0; i < count; ++i) {
        ivf_status st = check_csr(&X[i], k[i]);
        if (st != IVF_OK) return st;
    }
    ivf_options o;
    ivf_default_options(&o);
    if (opts) o = *opts;
    if (o.valtype < IVF_VAL_F32 || o.valtype > IVF_VAL_F16)
        return bfail(nullptr, IVF_ERR_ARG, "unknown valtype");
    ivf_batch* b = new (std::nothrow) ivf_batch();
    if (!b) return bfail(nullptr, IVF_ERR_OOM, "host allocation failed");
    auto bail = [&](ivf_status st) {
        const std::string msg = b->err;
        ivf_batch_destroy(b);
        g_build_error = msg;
        return st;
    };
    // a HIP failure while building: the batch is destroyed and the message kept
#define BUILD_HIP(call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return bail(bfail(b, e_ == hipErrorOutOfMemory ? IVF_ERR_OOM : IVF_ERR_HIP,  \
                              std::string(#call) + ": " + hipGetErrorString(e_)));       \
    } while (0)
    b->opt = o;
    // graph capture needs a stream of its own (never the null stream)
    if (o.stream) {
        b->stream = reinterpret_cast<hipStream_t>(o.stream);
    } else {
        BUILD_HIP(hipStreamCreate(&b->stream));
        b->own_stream = true;
    }
    b->opt.stream = b->stream;
    int dev = 0;
    BUILD_HIP(hipGetDevice(&dev));
    BUILD_HIP(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev));
    {
        std::vector<int32_t> order(count);
        for (int32_t i = 0; i < count; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t c) { return X[a].nnz > X[c].nnz; });
        int64_t load[ivf_batch::kLanes] = {};
        b->lane_of.assign(count, 0);
        for (int32_t i : order) {
            int best = 0;
            for (int l = 1; l < ivf_batch::kLanes; ++l)
                if (load[l] < load[best]) best = l;
            b->lane_of[i] = best;
            load[best] += X[i].nnz + 1;
        }
    }
    for (int l = 0; l < ivf_batch::kLanes; ++l) {
        BUILD_HIP(hipStreamCreate(&b->lane[l]));   // default priority
        BUILD_HIP(hipEventCreateWithFlags(&b->join_ev[l], hipEventDisableTiming));
        b->lane_sc[l] = new (std::nothrow) Scratch();
        if (!b->lane_sc[l]) return bail(bfail(b, IVF_ERR_OOM, "host allocation failed"));
        // a lane's scratch is sized for its largest instance up front
        int64_t maxnnz = 1;
        for (int32_t i = 0; i < count; ++i)
            if (b->lane_of[i] == l) maxnnz = std::max(maxnnz, X[i].nnz);
        BUILD_HIP(b->lane_sc[l]->ensure(maxnnz, maxnnz, 1, b->stream));
    }
    BUILD_HIP(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
    ivf_options oi = b->opt;
    oi.cluster_range = o.cluster_range > 0 ? o.cluster_range : 1280;
    oi.waves_per_wg = 1;
    for (int32_t i = 0; i < count; ++i) {
        ObjView* ov = nullptr;
        for (int32_t j = 0; j < i; ++j)   // instances on the same object set share its view
            if (X[j].indptr == X[i].indptr && X[j].indices == X[i].indices &&
                X[j].values == X[i].values && X[j].n == X[i].n && X[j].d == X[i].d &&
                X[j].nnz == X[i].nnz)
                ov = b->h[j]->ov;
        ivf_handle* h = nullptr;
        ivf_status st = create_handle(&X[i], k[i], oi, b->lane_sc[b->lane_of[i]], ov, &h);
        if (st != IVF_OK) return bail(bfail(b, st, g_build_error));
        h->owns_sc = false;
        if (!ov) {   // the batch owns every view; handles only borrow
            h->owns_ov = false;
            b->views.push_back(h->ov);
        }
        b->h.push_back(h);
    }
    BUILD_HIP(dalloc(&b->d_args, count));
    BUILD_HIP(dalloc(&b->d_item_off, count + 1));
    BUILD_HIP(dalloc(&b->d_flags, count));
    BUILD_HIP(dalloc(&b->d_cnt, count));
    {
        std::vector<Counters*> cp(count);
        for (int32_t i = 0; i < count; ++i) cp[i] = b->h[i]->cnt;
        BUILD_HIP(hipMemcpy(b->d_cnt, cp.data(), sizeof(Counters*) * count, hipMemcpyHostToDevice));
    }
    for (auto& e : b->ev) BUILD_HIP(hipEventCreate(&e));
    BUILD_HIP(dalloc(&b->d_stamp, 2));
    BUILD_HIP(dalloc(&b->d_work, 1));
    BUILD_HIP(hipDeviceGetAttribute(&b->clock_khz, hipDeviceAttributeWallClockRate, dev));
    if (b->clock_khz <= 0) return bail(bfail(b, IVF_ERR_HIP, "no device wall clock rate"));
    ivf_status st = batch_plan(b, oi.cluster_range, o.waves_per_wg > 0 ? o.waves_per_wg : 8);
    if (st != IVF_OK) return bail(st);
#undef BUILD_HIP
    *out = b;
    return IVF_OK;
}

ivf_status ivf_batch_init_seeds(ivf_batch* b, const int32_t* const* seeds) {
    if (!b || !seeds) return bfail(b, IVF_ERR_ARG, "null argument");
    for (size_t i = 0; i < b->h.size(); ++i) {
        ivf_status st = ivf_init_seeds(b->h[i], seeds[i]);
        if (st != IVF_OK) return bfail(b, st, b->h[i]->err);
    }
    return upload_args(b);
}

ivf_status ivf_batch_set_means(ivf_batch* b, int32_t inst, const ivf_means* M) {
    if (!b || inst < 0 || inst >= (int32_t)b->h.size()) return bfail(b, IVF_ERR_ARG, "bad instance");
    ivf_status st = ivf_set_means(b->h[inst], M);
    if (st != IVF_OK) return bfail(b, st, b->h[inst]->err);
    return upload_args(b);
}

ivf_status ivf_batch_iterate(ivf_batch* b, int32_t iters, int32_t* const* assign,
                             ivf_stats* stats) {
    if (!b || !assign || iters < 0) return bfail(b, IVF_ERR_ARG, "bad argument");
    const int32_t count = (int32_t)b->h.size();
    for (ivf_handle* h : b->h)
        if (!h->has_means) return bfail(b, IVF_ERR_STATE, "instance without means");
    for (int32_t r = 0; r < iters; ++r) {
        const bool eager = b->eager_left > 0;
        float ms = 0.f;
        if (eager) {
            for (ivf_handle* h : b->h) h->fixed = false;
            BHIP(b, hipEventRecord(b->ev[0], b->stream));
            ivf_status st = batch_iteration(b, assign, true);
            if (st != IVF_OK) return st;
            BHIP(b, hipEventRecord(b->ev[1], b->stream));
            BHIP(b, hipEventSynchronize(b->ev[1]));
            BHIP(b, hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
            if (--b->eager_left == 0) {
                if (!b->tuned && b->opt.cluster_range == 0) {
                    st = batch_autotune(b);
                    if (st != IVF_OK) return st;
                }
                st = batch_fix_capacities(b);
                if (st != IVF_OK) return st;
            }
        } else {
            bool same = b->exec[0] && b->exec[1] && b->captured_assign.size() == (size_t)count;
            for (int32_t i = 0; same && i < count; ++i) same = b->captured_assign[i] == assign[i];
            if (!same) {
                ivf_status st = batch_capture(b, assign);
                if (st != IVF_OK) return st;
            }
            BHIP(b, hipEventRecord(b->ev[0], b->stream));
            BHIP(b, hipGraphLaunch(b->exec[b->phase], b->stream));
            b->phase ^= 1;
            BHIP(b, hipEventRecord(b->ev[1], b->stream));
            for (ivf_handle* h : b->h) {
                h->cur = 1 - h->cur;
                h->nnzM_known = false;
            }
            k_gather_flags<<<(count + 63) / 64, 64, 0, b->stream>>>(b->d_cnt, count, b->d_flags);
            std::vector<unsigned long long> fl(count);
            BHIP(b, hipMemcpyAsync(fl.data(), b->d_flags, sizeof(unsigned long long) * count,
                                   hipMemcpyDeviceToHost, b->stream));
            BHIP(b, hipStreamSynchronize(b->stream));
            BHIP(b, hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
            // a fixed capacity was exceeded: the old means are intact, so that
            // update is redone eagerly with growth, then the graphs re-recorded
            bool redo = false;
            for (int32_t i = 0; i < count; ++i) {
                if (!(fl[i] & kOverflow)) continue;
                ivf_handle* h = b->h[i];
                h->cur = 1 - h->cur;
                h->fixed = false;
                // the update's own counters start again; the assignment's stay
                BHIP(b, hipMemsetAsync(&h->cnt->empty, 0, sizeof(unsigned long long), b->stream));
                BHIP(b, hipMemsetAsync(&h->cnt->error_flags, 0, sizeof(unsigned long long),
                                       b->stream));
                ivf_status st = run_update(h, assign[i], nullptr, false);
                if (st != IVF_OK) return bfail(b, st, h->err);
                redo = true;
            }
            if (redo) {
                ++b->recoveries;
                ivf_status st = batch_fix_capacities(b);
                if (st != IVF_OK) return st;
            }
        }
        if (stats) {
            BHIP(b, hipStreamSynchronize(b->stream));
            unsigned long long st[2] = {0, 0};
            BHIP(b, hipMemcpy(st, b->d_stamp, sizeof(st), hipMemcpyDeviceToHost));
            const float wms = (float)((double)(st[1] - st[0]) / (double)b->clock_khz);
            for (int32_t i = 0; i < count; ++i) {
                ivf_handle* h = b->h[i];
                ivf_stats* s = stats + (size_t)r * count + i;
                ivf_status st = assign_stats(h, s, false);
                if (st != IVF_OK) return bfail(b, st, h->err);
                double ds[2];
                Counters c;
                BHIP(b, hipMemcpy(ds, h->dscal, sizeof(ds), hipMemcpyDeviceToHost));
                BHIP(b, hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
                int64_t nnz_now = 0;
                BHIP(b, hipMemcpy(&nnz_now, h->mm_ptr[h->cur] + h->k, sizeof(int64_t),
                                  hipMemcpyDeviceToHost));
                s->objective_exact = ds[1];
                s->empty_clusters = (int64_t)c.empty;
                s->nnz_means = nnz_now;
                s->assign_ms = ms;    // the whole iteration of the batch
                s->walk_ms = wms;     // the one walk launch of the batch
                s->update_ms = 0.f;
            }
        }
    }
    BHIP(b, hipStreamSynchronize(b->stream));
    return IVF_OK;
}

ivf_status ivf_batch_get_means(ivf_batch* b, int32_t inst, ivf_means* out) {
    if (!b || inst < 0 || inst >= (int32_t)b->h.size()) return bfail(b, IVF_ERR_ARG, "bad instance");
    ivf_status st = ivf_get_means(b->h[inst], out);
    if (st != IVF_OK) return bfail(b, st, b->h[inst]->err);
    return IVF_OK;
}

ivf_status ivf_batch_set_slack(ivf_batch* b, double frac, int64_t abs_entries) {
    if (!b || !(frac >= 0.0) || frac > 64.0 || abs_entries < 0)
        return bfail(b, IVF_ERR_ARG, "slack must be 0 <= frac <= 64, abs >= 0");
    b->slack_frac = frac;
    b->slack_abs = abs_entries;
    if (b->eager_left == 0) return batch_fix_capacities(b);   // grows only
    return IVF_OK;
}

ivf_status ivf_batch_get_plan(const ivf_batch* b, int32_t plan[8]) {
    if (!b || !plan) return IVF_ERR_ARG;
    plan[0] = b->kr_max;
    plan[1] = b->waves;
    plan[2] = b->tile_stride;
    plan[3] = b->grid;
    plan[4] = (b->exec[0] && b->exec[1]) ? 1 : 0;
    plan[5] = b->tuned ? 1 : 0;
    plan[6] = b->captures;
    plan[7] = b->recoveries;
    return IVF_OK;
}

ivf_status ivf_batch_get_tuning(const ivf_batch* b, int32_t cap, int32_t* shapes, float* ms,
                                int32_t* count) {
    if (!b || !count || cap < 0 || (cap > 0 && (!shapes || !ms))) return IVF_ERR_ARG;
    const int32_t n = (int32_t)b->tune_ms.size();
    *count = n;
    for (int32_t i = 0; i < n && i < cap; ++i) {
        shapes[2 * i] = b->tune_shape[2 * i];
        shapes[2 * i + 1] = b->tune_shape[2 * i + 1];
        ms[i] = b->tune_ms[i];
    }
    return IVF_OK;
}

ivf_status ivf_batch_get_threshold_tuning(const ivf_batch* b, int32_t cap, float* thetas,
                                          float* ms, int32_t* count) {
    if (!b || !count || cap < 0 || (cap > 0 && (!thetas || !ms))) return IVF_ERR_ARG;
    const int32_t n = (int32_t)b->tune_theta.size();
    *count = n;
    for (int32_t i = 0; i < n && i < cap; ++i) {
        thetas[i] = b->tune_theta[i];
        ms[i] = b->tune_theta_ms[i];
    }
    return IVF_OK;
}

void ivf_batch_destroy(ivf_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (int l = 0; l < ivf_batch::kLanes; ++l)
        if (b->lane[l]) (void)hipStreamSynchronize(b->lane[l]);
    drop_graphs(b);
    for (ivf_handle* h : b->h) {
        free_handle(h);
        delete h;
    }
    for (ObjView* v : b->views) {
        v->release();
        delete v;
    }
    for (int l = 0; l < ivf_batch::kLanes; ++l) {
        if (b->lane[l]) (void)hipStreamSynchronize(b->lane[l]);
        if (b->lane_sc[l]) { b->lane_sc[l]->release(); delete b->lane_sc[l]; }
        if (b->lane[l]) (void)hipStreamDestroy(b->lane[l]);
        if (b->join_ev[l]) (void)hipEventDestroy(b->join_ev[l]);
    }
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    dfree(b->d_args);
    dfree(b->d_item_off);
    dfree(b->d_flags);
    dfree(b->d_cnt);
    for (auto& e : b->ev)
        if (e) (void)hipEventDestroy(e);
    dfree(b->d_stamp);
    dfree(b->d_work);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char* ivf_batch_last_error(const ivf_batch* b) {
    return b ? b->err.c_str() : g_build_error.c_str();
}

}  // extern "C"
