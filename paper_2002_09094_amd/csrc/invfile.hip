// The inverted file of the means (Algorithm 3's M-breve) for gfx950: term t
// -> its list of (cluster j, mean value) in ascending j, rebuilt after every
// update, with the layout the assignment walk reads.
//
// A stable radix sort of the new mean-major entries by term leaves every
// term's list in ascending cluster order, the order the paper's update loop
// produces.  Per (term, cluster range) a slice descriptor then names either
// the sparse entries of the list that fall in the range or, where the term
// covers at least a threshold share of the range's clusters, a dense slab of
// the range's width (zeros for absent clusters, 128-byte aligned): the
// paper's IFN layout applied per slice.
#include "ivf_internal.h"
#include "kernels.h"

namespace ivf {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b > 0 ? b : 1);
}

inline unsigned capped(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

inline int bits_for(int64_t maxval) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) <= maxval) ++b;
    return b;
}

#define HIP_RET(x)                           \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

__device__ inline int64_t lower_bound_i32(const int32_t* a, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Sort keys and payload of every mean entry (the first n_dev of n when
// given): its term, and its cluster with the FP32 rounding of its value.
__global__ void k_term_entries(const int32_t* __restrict__ mm_idx,
                               const int32_t* __restrict__ mm_row,
                               const double* __restrict__ mm_val, int64_t n, const int64_t* n_dev,
                               uint32_t* __restrict__ keys, uint2* __restrict__ pay) {
    n = bounded_count(n, n_dev);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        keys[e] = (uint32_t)mm_idx[e];
        pay[e] = make_uint2((uint32_t)mm_row[e], __float_as_uint((float)mm_val[e]));
    }
}

__device__ inline uint32_t bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// The sorted entries as postings in the stored precision: FP32 {cluster,
// value}; 16-bit {local cluster id | value << 16}; and each entry's cluster.
__global__ void k_ivf_store(const uint2* __restrict__ pay, int64_t nnzM, const int64_t* n_dev,
                            int32_t k_r, int valtype, int32_t* __restrict__ cid,
                            void* __restrict__ post) {
    nnzM = bounded_count(nnzM, n_dev);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnzM;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint2 e = pay[q];
        const int32_t j = (int32_t)e.x;
        cid[q] = j;
        if (valtype == IVF_VAL_F32) {
            reinterpret_cast<uint2*>(post)[q] = e;
        } else {
            const float f = __uint_as_float(e.y);
            const uint32_t local = (uint32_t)(j % k_r);
            uint32_t h;
            if (valtype == IVF_VAL_BF16) h = bf16_rne(f);
            else h = (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)f);
            reinterpret_cast<uint32_t*>(post)[q] = local | (h << 16);
        }
    }
}

__global__ void k_ivf_ptr(const uint32_t* skeys, int64_t nnzM, const int64_t* n_dev, int64_t d,
                          int64_t* ptr) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > d) return;
    nnzM = bounded_count(nnzM, n_dev);
    int64_t lo = 0, hi = nnzM;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (skeys[mid] < (uint32_t)t) lo = mid + 1; else hi = mid;
    }
    ptr[t] = lo;
}

// Per (term, range) slice: sparse start and count; dense slab size when the
// slice holds at least `theta` of the range's clusters.
__global__ void k_desc(const int64_t* ptr, const int32_t* cid, int64_t d, int32_t k, int32_t R,
                       int32_t k_r, float theta, int32_t align, SliceDesc* desc, int64_t* dsz) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d) {
        if (t == d) dsz[d * R] = 0;
        return;
    }
    const int64_t a = ptr[t], b = ptr[t + 1];
    int64_t lo = a;
    for (int32_t r = 0; r < R; ++r) {
        const int64_t hi = lower_bound_i32(cid, lo, b, (r + 1) * k_r);
        const int64_t cnt = hi - lo;
        const int32_t kr = min(k_r, k - r * k_r);
        SliceDesc ds;
        ds.pos = (int32_t)lo;
        ds.count = (int32_t)cnt;
        desc[t * R + r] = ds;
        // a dense slab's size is rounded up to whole 128-byte lines, so every
        // slab starts on a line (0.5-0.8 % faster walks at 8M documents); the
        // sizes are laid out range-major, so a range's slabs are contiguous
        dsz[(int64_t)r * d + t] = (cnt > 0 && (float)cnt >= theta * (float)kr)
                             ? (int64_t)((kr + align - 1) / align * align)
                             : 0;
        lo = hi;
    }
}

__global__ void k_desc_dense(SliceDesc* desc, const int64_t* doff, int64_t d, int32_t R,
                             int64_t cap) {
    // slice (t, r) is desc[t * R + r], its scanned slab offset doff[r * d + t];
    // a slice is dense iff that offset grows to the next entry; one that would
    // not fit the slab capacity stays sparse (same scores)
    const int64_t nslices = d * R;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslices;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = (s % R) * d + s / R;
        if (doff[o + 1] > doff[o] && doff[o + 1] <= cap) desc[s].pos = (int32_t)(-(doff[o] + 1));
    }
}

template <typename T>
__global__ void k_zero_t(T* p, int64_t n, const int64_t* n_dev = nullptr) {
    if (n_dev) n = min(n, *n_dev);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// Dense slabs take every entry of their slice at its cluster's offset.
__global__ void k_slab_scatter(const uint32_t* __restrict__ skeys, const int32_t* __restrict__ cid,
                               const void* __restrict__ post, const SliceDesc* __restrict__ desc,
                               int64_t nnzM, const int64_t* n_dev, int64_t d, int32_t k,
                               int32_t R, int32_t k_r, int valtype, void* __restrict__ slab) {
    nnzM = bounded_count(nnzM, n_dev);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnzM;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = skeys[q];
        const int32_t j = cid[q];
        if (t >= d || j < 0 || j >= k) continue;   // never true for validated means
        const int32_t r = j / k_r;
        const int64_t pos = desc[t * R + r].pos;
        if (pos >= 0) continue;
        const int64_t at = (-pos - 1) + (j - r * k_r);
        if (valtype == IVF_VAL_F32)
            reinterpret_cast<float*>(slab)[at] =
                __uint_as_float(reinterpret_cast<const uint2*>(post)[q].y);
        else
            reinterpret_cast<uint16_t*>(slab)[at] =
                (uint16_t)(reinterpret_cast<const uint32_t*>(post)[q] >> 16);
    }
}

}  // namespace

hipError_t launch_build_ivf(IvfArgs& a, hipStream_t s) {
    // a.nnzM: the entry count, or the capacity when a.nnz_dev holds the count
    if (a.nnzM > 0) {
        // stable by term: lists in ascending cluster order, the entries' payload
        // moving with them (no gather through positions afterwards)
        k_term_entries<<<capped(a.nnzM), kThreads, 0, s>>>(a.mm_idx, a.mm_row, a.mm_val, a.nnzM,
                                                          a.nnz_dev, a.keys, a.pay);
        HIP_RET(hipGetLastError());
        HIP_RET(radix_sort_pairs_u64(a.keys, a.pay, a.keys_alt, a.pay_alt, a.nnzM,
                                     bits_for(a.d - 1 > 0 ? a.d - 1 : 1), a.tmp, s, nullptr,
                                     a.nnz_dev));
        k_ivf_store<<<capped(a.nnzM), kThreads, 0, s>>>(a.pay, a.nnzM, a.nnz_dev, a.k_r,
                                                       a.valtype, a.cid, a.post);
        HIP_RET(hipGetLastError());
    }
    k_ivf_ptr<<<grid_for(a.d + 1), kThreads, 0, s>>>(a.keys, a.nnzM, a.nnz_dev, a.d, a.ivf_ptr);
    k_desc<<<grid_for(a.d + 1), kThreads, 0, s>>>(a.ivf_ptr, a.cid, a.d, a.k, a.R, a.k_r,
                                                  a.dense_threshold,
                                                  a.valtype == IVF_VAL_F32 ? 32 : 64, a.desc, a.dsz);
    HIP_RET(hipGetLastError());
    return exclusive_scan_i64(a.dsz, a.dsz, a.d * a.R + 1, a.tmp, s);
}

hipError_t launch_build_slabs(IvfArgs& a, int64_t slab_cap, hipStream_t s) {
    // slab_cap: elements the slab array holds; the needed total is at dsz[d * R]
    const int64_t ns = a.d * a.R;
    if (slab_cap <= 0) return hipSuccess;
    k_desc_dense<<<capped(ns), kThreads, 0, s>>>(a.desc, a.dsz, a.d, a.R, slab_cap);
    const int64_t* total = a.dsz + ns;
    if (a.valtype == IVF_VAL_F32)
        k_zero_t<float><<<capped(slab_cap), kThreads, 0, s>>>(reinterpret_cast<float*>(a.slab),
                                                               slab_cap, total);
    else
        k_zero_t<uint16_t><<<capped(slab_cap), kThreads, 0, s>>>(
            reinterpret_cast<uint16_t*>(a.slab), slab_cap, total);
    if (a.nnzM > 0)
        k_slab_scatter<<<capped(a.nnzM), kThreads, 0, s>>>(a.keys, a.cid, a.post, a.desc, a.nnzM,
                                                           a.nnz_dev, a.d, a.k, a.R, a.k_r,
                                                           a.valtype, a.slab);
    return hipGetLastError();
}

}  // namespace ivf
