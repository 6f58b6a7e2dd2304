// C ABI of the library (declared in include/ivf.h): handle, validation,
// planning, memory and the order of launches for one Lloyd iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "ivf_internal.h"
#include "kernels.h"

using namespace ivf;

struct ivf_handle {
    // configuration
    int64_t n = 0, d = 0, nnz = 0;
    int32_t k = 0;
    ivf_options opt{};
    hipStream_t stream = nullptr;
    Plan plan;
    int device = 0, cus = 0;
    int walk_grid = 0, rescore_grid = 0;
    // objects (borrowed)
    const int64_t* x_ptr = nullptr;
    const int32_t* x_idx = nullptr;
    const float* x_val = nullptr;
    // term-major view of the objects
    int32_t* xt_obj = nullptr;
    int32_t* xt_term = nullptr;
    float* xt_val = nullptr;
    int16_t* shift = nullptr;
    int64_t inexact_terms = 0;
    // sort / segment scratch
    int64_t sort_cap = 0;
    uint32_t *keys = nullptr, *vals = nullptr, *keys_alt = nullptr, *vals_alt = nullptr;
    uint32_t* iota = nullptr;
    uint32_t *flag = nullptr, *segpos = nullptr;
    unsigned long long* seg_acc = nullptr;
    int32_t *seg_j = nullptr, *seg_t = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    // clusters
    int64_t *size = nullptr, *cstart = nullptr, *newcnt = nullptr, *scal = nullptr;
    double *nrm = nullptr, *objpart = nullptr;
    // means, mean-major FP64, double-buffered
    int cur = 0;
    bool has_means = false;
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
    void* slab = nullptr;
    int64_t slab_cap = 0;     // bytes
    int64_t slab_elems = 0;
    int32_t* cid = nullptr;
    double* val64 = nullptr;
    void* post = nullptr;
    // assignment scratch
    RangeRec* rec = nullptr;
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
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    std::string err;
};

namespace {

constexpr int kObjBlocks = 1024;
thread_local std::string g_build_error;

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

void free_all(ivf_handle* h) {
    dfree(h->xt_obj); dfree(h->xt_term); dfree(h->xt_val); dfree(h->shift);
    dfree(h->keys); dfree(h->vals); dfree(h->keys_alt); dfree(h->vals_alt); dfree(h->iota);
    dfree(h->flag); dfree(h->segpos); dfree(h->seg_acc); dfree(h->seg_j); dfree(h->seg_t);
    if (h->tmp) (void)hipFree(h->tmp);
    h->tmp = nullptr;
    dfree(h->size); dfree(h->cstart); dfree(h->newcnt); dfree(h->scal);
    dfree(h->nrm); dfree(h->objpart);
    for (int b = 0; b < 2; ++b) {
        dfree(h->mm_ptr[b]); dfree(h->mm_idx[b]); dfree(h->mm_val[b]); dfree(h->mm_row[b]);
    }
    dfree(h->ivf_ptr); dfree(h->desc); dfree(h->dsz); dfree(h->cid); dfree(h->val64);
    if (h->slab) (void)hipFree(h->slab);
    h->slab = nullptr;
    if (h->post) (void)hipFree(h->post);
    h->post = nullptr;
    dfree(h->rec); dfree(h->prev); dfree(h->seed_assign); dfree(h->rho); dfree(h->best);
    dfree(h->second); dfree(h->best_id); dfree(h->flags); dfree(h->rescore_list);
    dfree(h->part); dfree(h->dscal); dfree(h->cnt);
    for (auto& e : h->ev)
        if (e) { (void)hipEventDestroy(e); e = nullptr; }
}

// Sort buffers and scan/sort scratch sized for `need` elements.
ivf_status ensure_sort(ivf_handle* h, int64_t need) {
    if (need <= h->sort_cap) return IVF_OK;
    const int64_t cap = std::max<int64_t>(need, h->sort_cap + h->sort_cap / 4);
    dfree(h->keys); dfree(h->vals); dfree(h->keys_alt); dfree(h->vals_alt); dfree(h->iota);
    if (h->tmp) (void)hipFree(h->tmp);
    h->tmp = nullptr;
    HIPCHK(h, dalloc(&h->keys, cap));
    HIPCHK(h, dalloc(&h->vals, cap));
    HIPCHK(h, dalloc(&h->keys_alt, cap));
    HIPCHK(h, dalloc(&h->vals_alt, cap));
    HIPCHK(h, dalloc(&h->iota, cap));
    const int64_t scan_n = std::max<int64_t>(std::max<int64_t>(cap, (int64_t)h->k + 1),
                                             h->d * (int64_t)h->plan.R + 1);
    h->tmp_bytes = std::max(radix_tmp_bytes(cap), scan_tmp_bytes(scan_n));
    HIPCHK(h, hipMalloc(&h->tmp, h->tmp_bytes));
    HIPCHK(h, launch_iota(h->iota, cap, h->stream));
    h->sort_cap = cap;
    return IVF_OK;
}

ivf_status ensure_mm(ivf_handle* h, int b, int64_t need) {
    if (need <= h->mm_cap[b]) return IVF_OK;
    const int64_t cap = std::max<int64_t>(need, h->mm_cap[b] + h->mm_cap[b] / 4);
    dfree(h->mm_idx[b]); dfree(h->mm_val[b]); dfree(h->mm_row[b]);
    HIPCHK(h, dalloc(&h->mm_idx[b], cap));
    HIPCHK(h, dalloc(&h->mm_val[b], cap));
    HIPCHK(h, dalloc(&h->mm_row[b], cap));
    h->mm_cap[b] = cap;
    return IVF_OK;
}

ivf_status ensure_ivf(ivf_handle* h, int64_t need) {
    if (need > h->ivf_cap) {
        const int64_t cap = std::max<int64_t>(need, h->ivf_cap + h->ivf_cap / 4);
        dfree(h->cid); dfree(h->val64);
        if (h->post) (void)hipFree(h->post);
        h->post = nullptr;
        HIPCHK(h, dalloc(&h->cid, cap));
        HIPCHK(h, dalloc(&h->val64, cap));
        HIPCHK(h, hipMalloc(&h->post, (size_t)std::max<int64_t>(cap, 1) * 8));
        h->ivf_cap = cap;
    }
    return ensure_sort(h, need);
}

ivf_status read_errors(ivf_handle* h, const char* what) {
    Counters c;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
    const unsigned long long f = c.error_flags;
    if (!f) return IVF_OK;
    std::string m = std::string(what) + ": ";
    if (f & kBadPtr) return fail(h, IVF_ERR_ARG, m + "row pointers inconsistent with sizes");
    if (f & kBadIndex) return fail(h, IVF_ERR_UNSORTED, m + "term id outside [0, d)");
    if (f & kBadOrder) return fail(h, IVF_ERR_UNSORTED, m + "term ids not strictly ascending");
    if (f & kNonFinite) return fail(h, IVF_ERR_NONFINITE, m + "non-finite value");
    return fail(h, IVF_ERR_NEGATIVE, m + "value <= 0");
}

// Rebuild the inverted file from mean-major buffer `b` holding nnzM entries.
ivf_status rebuild_ivf(ivf_handle* h, int b, int64_t nnzM) {
    ivf_status st = ensure_ivf(h, nnzM);
    if (st != IVF_OK) return st;
    IvfArgs a{};
    a.d = h->d;
    a.nnzM = nnzM;
    a.k = h->k;
    a.k_r = h->plan.k_r;
    a.R = h->plan.R;
    a.valtype = h->opt.valtype;
    a.dense_threshold = h->opt.dense_threshold > 0.f ? h->opt.dense_threshold : 0.5f;
    a.mm_idx = h->mm_idx[b];
    a.mm_val = h->mm_val[b];
    a.mm_row = h->mm_row[b];
    a.keys = h->keys;
    a.vals = h->vals;
    a.keys_alt = h->keys_alt;
    a.vals_alt = h->vals_alt;
    a.iota = h->iota;
    a.ivf_ptr = h->ivf_ptr;
    a.desc = h->desc;
    a.dsz = h->dsz;
    a.cid = h->cid;
    a.val64 = h->val64;
    a.post = h->post;
    a.tmp = h->tmp;
    HIPCHK(h, launch_build_ivf(a, h->stream));
    // size the dense slabs (the scanned total) before filling them
    int64_t elems = 0;
    HIPCHK(h, hipMemcpyAsync(&elems, h->dsz + h->d * h->plan.R, sizeof(int64_t),
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const int64_t bytes = elems * (h->opt.valtype == IVF_VAL_F32 ? 4 : 2);
    if (bytes > h->slab_cap) {
        if (h->slab) (void)hipFree(h->slab);
        h->slab = nullptr;
        h->slab_cap = 0;
        const int64_t cap = std::max<int64_t>(bytes, bytes + bytes / 4);
        HIPCHK(h, hipMalloc(&h->slab, (size_t)cap));
        h->slab_cap = cap;
    }
    a.slab = h->slab;
    HIPCHK(h, launch_build_slabs(a, elems, h->stream));
    h->slab_elems = elems;
    return IVF_OK;
}

// Update step from `assign`: new means into buffer 1 - cur, then the swap and
// the inverted-file rebuild.
ivf_status run_update(ivf_handle* h, const int32_t* assign, ivf_stats* stats) {
    const hipStream_t s = h->stream;
    if (stats) HIPCHK(h, hipEventRecord(h->ev[2], s));
    HIPCHK(h, launch_clear_counters(h->cnt, s));
    const int o = h->cur, nb = 1 - h->cur;
    UpdateArgs a{};
    a.n = h->n; a.d = h->d; a.nnz = h->nnz; a.k = h->k;
    a.assign = assign;
    a.xt_obj = h->xt_obj; a.xt_term = h->xt_term; a.xt_val = h->xt_val; a.shift = h->shift;
    a.keys = h->keys; a.vals = h->vals; a.keys_alt = h->keys_alt; a.vals_alt = h->vals_alt;
    a.iota = h->iota;
    a.flag = h->flag; a.segpos = h->segpos; a.seg_acc = h->seg_acc;
    a.seg_j = h->seg_j; a.seg_t = h->seg_t;
    a.size = h->size; a.cstart = h->cstart; a.nrm = h->nrm; a.objpart = h->objpart;
    a.newcnt = h->newcnt; a.scal = h->scal;
    a.old_ptr = h->mm_ptr[o]; a.old_idx = h->mm_idx[o]; a.old_val = h->mm_val[o];
    a.new_ptr = h->mm_ptr[nb];
    a.cnt = h->cnt;
    a.tmp = h->tmp;
    HIPCHK(h, launch_update_sums(a, s));
    int64_t nnz_new = 0;
    HIPCHK(h, hipMemcpyAsync(&nnz_new, h->mm_ptr[nb] + h->k, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    ivf_status st = ensure_mm(h, nb, nnz_new);
    if (st != IVF_OK) return st;
    a.new_idx = h->mm_idx[nb];
    a.new_val = h->mm_val[nb];
    a.new_row = h->mm_row[nb];
    HIPCHK(h, launch_update_fill(a, s));
    HIPCHK(h, launch_objective_exact(h->objpart, h->k, h->dscal + 1, s));
    st = rebuild_ivf(h, nb, nnz_new);
    if (st != IVF_OK) return st;
    h->cur = nb;
    h->nnzM = nnz_new;
    h->has_means = true;
    if (stats) {
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
        stats->inexact_terms = h->inexact_terms;
        stats->update_ms = ms;
    }
    return IVF_OK;
}

}  // namespace

// ------------------------------------------------------------------- planner
namespace ivf {

ivf_status make_plan(int32_t k, const ivf_options* o, Plan* p, std::string* err) {
    if (k < 1) {
        if (err) *err = "k must be >= 1";
        return IVF_ERR_ARG;
    }
    // 1280 clusters per tile and 8 tiles per workgroup (40 KB of LDS, 4
    // workgroups and 32 waves per CU) measured best at 8M documents x k = 10,000
    int32_t kr_max = (o && o->cluster_range > 0) ? o->cluster_range : 1280;
    if (kr_max > 32768) {
        if (err) *err = "cluster_range above 32768 (LDS tile and 16-bit local ids)";
        return IVF_ERR_ARG;
    }
    const bool forced_waves = o && o->waves_per_wg > 0;
    int32_t waves = forced_waves ? o->waves_per_wg : 8;
    if (waves > kMaxWaves) {
        if (err) *err = "waves_per_wg above 16";
        return IVF_ERR_ARG;
    }
    Plan q;
    q.k = k;
    q.R = (k + kr_max - 1) / kr_max;
    q.k_r = (k + q.R - 1) / q.R;
    q.tile_stride = (q.k_r + 3) & ~3;
    while (!forced_waves && waves > 1 && (int64_t)waves * q.tile_stride * 4 > kLdsBytes) --waves;
    q.waves = waves;
    q.lds_bytes = waves * q.tile_stride * 4;
    if (q.lds_bytes > kLdsBytes) {
        if (err) *err = "score tiles exceed the 160 KB LDS";
        return IVF_ERR_ARG;
    }
    q.chunk = (o && o->objects_per_item > 0) ? o->objects_per_item : (q.k_r >= 1024 ? 1 : 8);
    q.k_r64 = std::min<int32_t>(k, 8192);
    q.R64 = (k + q.k_r64 - 1) / q.k_r64;
    *p = q;
    return IVF_OK;
}

}  // namespace ivf

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

ivf_status ivf_cert_bound(int32_t valtype, int64_t nt, double c[3]) {
    if (!c || valtype < IVF_VAL_F32 || valtype > IVF_VAL_F16 || nt < 0) return IVF_ERR_ARG;
    cert_consts(valtype, nt, &c[0], &c[1], &c[2]);
    return IVF_OK;
}

ivf_status ivf_build(const ivf_csr* X, int32_t k, const ivf_options* opts, ivf_handle** out) {
    if (out) *out = nullptr;
    if (!X || !out) return fail(nullptr, IVF_ERR_ARG, "null argument");
    if (X->n < 1 || X->d < 1 || X->nnz < 0) return fail(nullptr, IVF_ERR_ARG, "bad sizes");
    if (!X->indptr || (X->nnz > 0 && (!X->indices || !X->values)))
        return fail(nullptr, IVF_ERR_ARG, "null object arrays");
    if (k < 1 || (int64_t)k > X->n) return fail(nullptr, IVF_ERR_ARG, "k outside [1, n]");
    if (k >= (1 << 24)) return fail(nullptr, IVF_ERR_CAPACITY, "k >= 2^24");
    if (X->nnz >= ((int64_t)1 << 31) - 1 || X->n >= ((int64_t)1 << 31) - 1 ||
        X->d >= ((int64_t)1 << 31) - 1)
        return fail(nullptr, IVF_ERR_CAPACITY, "n, d or nnz >= 2^31");
    ivf_options o;
    ivf_default_options(&o);
    if (opts) o = *opts;
    if (o.valtype < IVF_VAL_F32 || o.valtype > IVF_VAL_F16)
        return fail(nullptr, IVF_ERR_ARG, "unknown valtype");
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
    h->x_ptr = X->indptr; h->x_idx = X->indices; h->x_val = X->values;
    auto bail = [&](ivf_status st) {
        g_build_error = h->err;
        free_all(h);
        delete h;
        return st;
    };
#define BCHK(call)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bail(fail(h, e_ == hipErrorOutOfMemory ? IVF_ERR_OOM : IVF_ERR_HIP,     \
                             std::string(#call) + ": " + hipGetErrorString(e_)));          \
    } while (0)
#define BST(expr)                            \
    do {                                     \
        ivf_status s_ = (expr);              \
        if (s_ != IVF_OK) return bail(s_);   \
    } while (0)

    BCHK(hipGetDevice(&h->device));
    BCHK(hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device));
    for (auto& e : h->ev) BCHK(hipEventCreate(&e));
    BCHK(dalloc(&h->cnt, 1));
    BCHK(launch_clear_counters(h->cnt, h->stream));
    // validation before anything else reads the objects
    ObjectView xv{X->indptr, X->indices, X->values, X->n, X->d, X->nnz};
    BCHK(launch_validate_objects(xv, h->cnt, h->stream));
    BST(read_errors(h, "objects"));

    const int64_t n = h->n, d = h->d, nnz = h->nnz;
    BST(ensure_sort(h, std::max<int64_t>(nnz, 1)));
    // term-major view: stable sort of (term, position), positions ascend with objects
    int32_t* rowid = nullptr;
    BCHK(dalloc(&rowid, nnz));
    BCHK(dalloc(&h->xt_obj, nnz));
    BCHK(dalloc(&h->xt_term, nnz));
    BCHK(dalloc(&h->xt_val, nnz));
    if (nnz > 0) {
        BCHK(launch_row_ids(X->indptr, n, rowid, h->stream));
        BCHK(launch_copy_keys(X->indices, h->keys, nnz, h->stream));
        int bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) <= d - 1) ++bits;
        BCHK(radix_sort_pairs(h->keys, h->vals, h->keys_alt, h->vals_alt, nnz, bits, h->tmp,
                              h->stream, h->iota));
        BCHK(launch_build_xt(h->keys, h->vals, rowid, X->values, nnz, h->xt_obj, h->xt_term,
                             h->xt_val, h->stream));
    }
    // per-term fixed-point scales of the member sums
    int32_t *emin = nullptr, *emax = nullptr, *tcount = nullptr;
    BCHK(dalloc(&emin, d));
    BCHK(dalloc(&emax, d));
    BCHK(dalloc(&tcount, d));
    BCHK(dalloc(&h->shift, d));
    BCHK(launch_term_shift(X->indices, X->values, nnz, d, emin, emax, tcount, h->shift, h->cnt,
                           h->stream));
    {
        Counters c;
        BCHK(hipStreamSynchronize(h->stream));
        BCHK(hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
        h->inexact_terms = (int64_t)c.pad[0];
    }
    (void)hipFree(rowid);
    (void)hipFree(emin);
    (void)hipFree(emax);
    (void)hipFree(tcount);
    // segment and cluster scratch
    BCHK(dalloc(&h->flag, nnz));
    BCHK(dalloc(&h->segpos, nnz));
    BCHK(dalloc(&h->seg_acc, nnz));
    BCHK(dalloc(&h->seg_j, nnz));
    BCHK(dalloc(&h->seg_t, nnz));
    BCHK(dalloc(&h->size, k));
    BCHK(dalloc(&h->cstart, (int64_t)k + 1));
    BCHK(dalloc(&h->newcnt, (int64_t)k + 1));
    BCHK(dalloc(&h->scal, 4));
    BCHK(dalloc(&h->nrm, k));
    BCHK(dalloc(&h->objpart, k));
    for (int b = 0; b < 2; ++b) {
        BCHK(dalloc(&h->mm_ptr[b], (int64_t)k + 1));
        BCHK(hipMemsetAsync(h->mm_ptr[b], 0, sizeof(int64_t) * ((size_t)k + 1), h->stream));
    }
    BST(ensure_mm(h, 0, 1));
    BST(ensure_mm(h, 1, 1));
    BCHK(dalloc(&h->ivf_ptr, d + 1));
    BCHK(dalloc(&h->desc, d * (int64_t)plan.R));
    BCHK(dalloc(&h->dsz, d * (int64_t)plan.R + 1));
    BST(ensure_ivf(h, 1));
    // assignment scratch
    BCHK(dalloc(&h->rec, n * (int64_t)plan.R));
    BCHK(dalloc(&h->prev, n));
    BCHK(dalloc(&h->seed_assign, n));
    BCHK(dalloc(&h->rho, n));
    BCHK(dalloc(&h->best, n));
    BCHK(dalloc(&h->second, n));
    BCHK(dalloc(&h->best_id, n));
    BCHK(dalloc(&h->flags, n));
    BCHK(dalloc(&h->rescore_list, n));
    BCHK(dalloc(&h->part, kObjBlocks));
    BCHK(dalloc(&h->dscal, 4));
    // launch shapes
    BCHK(walk_set_lds_limit(std::max(plan.lds_bytes, 1)));
    int per_cu = 0;
    BCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, walk_kernel_ptr(o.valtype), kWave * plan.waves,
        (size_t)plan.lds_bytes));
    if (per_cu < 1) per_cu = 1;
    h->walk_grid = h->cus * per_cu;
    h->rescore_grid = h->cus * 2;
    BCHK(hipStreamSynchronize(h->stream));
#undef BCHK
#undef BST
    *out = h;
    return IVF_OK;
}

void ivf_destroy(ivf_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
}

ivf_status ivf_set_means(ivf_handle* h, const ivf_means* M) {
    if (!h || !M) return fail(h, IVF_ERR_ARG, "null argument");
    if (M->k != h->k || M->d != h->d || M->nnz < 0)
        return fail(h, IVF_ERR_ARG, "means k/d do not match the handle");
    if (!M->indptr || (M->nnz > 0 && (!M->indices || !M->values)))
        return fail(h, IVF_ERR_ARG, "null mean arrays");
    if (M->nnz >= ((int64_t)1 << 31) - 1) return fail(h, IVF_ERR_CAPACITY, "nnz >= 2^31");
    HIPCHK(h, launch_clear_counters(h->cnt, h->stream));
    HIPCHK(h, launch_validate_means(M->indptr, M->indices, M->values, h->k, h->d, M->nnz, h->cnt,
                                    h->stream));
    ivf_status st = read_errors(h, "means");
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
    st = rebuild_ivf(h, b, M->nnz);
    if (st != IVF_OK) return st;
    h->nnzM = M->nnz;
    h->has_means = true;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return IVF_OK;
}

ivf_status ivf_init_seeds(ivf_handle* h, const int32_t* seeds) {
    if (!h || !seeds) return fail(h, IVF_ERR_ARG, "null argument");
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
    const hipStream_t s = h->stream;
    const Plan& p = h->plan;
    if (stats) HIPCHK(h, hipEventRecord(h->ev[0], s));
    HIPCHK(h, launch_clear_counters(h->cnt, s));
    HIPCHK(h, hipMemcpyAsync(h->prev, assign, sizeof(int32_t) * (size_t)h->n,
                             hipMemcpyDeviceToDevice, s));
    WalkArgs w{};
    w.x_ptr = h->x_ptr; w.x_idx = h->x_idx; w.x_val = h->x_val; w.n = h->n;
    w.desc = h->desc; w.post = h->post; w.slab = h->slab;
    w.k = h->k; w.k_r = p.k_r; w.R = p.R; w.chunk = p.chunk; w.tile_stride = p.tile_stride;
    w.items_per_range = (h->n + p.chunk - 1) / p.chunk;
    w.cnt = h->cnt; w.rec = h->rec;
    if (stats) HIPCHK(h, hipEventRecord(h->ev[4], s));
    HIPCHK(h, launch_walk(w, h->opt.valtype, p.waves, p.lds_bytes, h->walk_grid, s));
    if (stats) HIPCHK(h, hipEventRecord(h->ev[5], s));
    MergeArgs m{};
    m.x_ptr = h->x_ptr; m.n = h->n; m.R = p.R;
    m.valtype = h->opt.valtype; m.certify = h->opt.certify; m.force_rescore = h->opt.force_rescore;
    m.rec = h->rec; m.prev = h->prev; m.assign = assign; m.rho = h->rho;
    m.best = h->best; m.best_id = h->best_id; m.second = h->second; m.flags = h->flags;
    m.rescore_list = h->rescore_list; m.cnt = h->cnt;
    HIPCHK(h, launch_merge(m, s));
    if (h->opt.certify) {
        RescoreArgs r{};
        r.x_ptr = h->x_ptr; r.x_idx = h->x_idx; r.x_val = h->x_val;
        r.ivf_ptr = h->ivf_ptr; r.cid = h->cid; r.val64 = h->val64;
        r.k = h->k; r.k_r64 = p.k_r64; r.R64 = p.R64;
        r.rescore_list = h->rescore_list; r.prev = h->prev; r.assign = assign; r.rho = h->rho;
        r.best = h->best; r.best_id = h->best_id; r.cnt = h->cnt;
        HIPCHK(h, launch_rescore(r, h->rescore_grid, s));
    }
    HIPCHK(h, launch_objective(h->rho, assign, h->prev, h->n, h->part, kObjBlocks, h->dscal, h->cnt,
                               s));
    if (stats) {
        HIPCHK(h, hipEventRecord(h->ev[1], s));
        HIPCHK(h, hipStreamSynchronize(s));
        Counters c;
        double obj = 0.0;
        HIPCHK(h, hipMemcpy(&c, h->cnt, sizeof(c), hipMemcpyDeviceToHost));
        HIPCHK(h, hipMemcpy(&obj, h->dscal, sizeof(obj), hipMemcpyDeviceToHost));
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
        float wms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&wms, h->ev[4], h->ev[5]));
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
        stats->max_rel_err = err;
        stats->assign_ms = ms;
        stats->walk_ms = wms;
        stats->objective_exact = std::nan("");
        stats->empty_clusters = -1;
        stats->nnz_means = h->nnzM;
        stats->inexact_terms = h->inexact_terms;
        stats->update_ms = 0.f;
    }
    return IVF_OK;
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

ivf_status ivf_get_means(ivf_handle* h, ivf_means* out) {
    if (!h || !out) return fail(h, IVF_ERR_ARG, "null argument");
    if (!h->has_means) return fail(h, IVF_ERR_STATE, "no means yet");
    out->k = h->k;
    out->d = h->d;
    if (!out->indptr) {
        out->nnz = h->nnzM;
        return IVF_OK;
    }
    if (out->nnz < h->nnzM || (h->nnzM > 0 && (!out->indices || !out->values)))
        return fail(h, IVF_ERR_ARG, "output buffers smaller than nnz");
    const int b = h->cur;
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

}  // extern "C"
