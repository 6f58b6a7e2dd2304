// Update step of inverted-file spherical k-means (Algorithm 3, update part)
// and the inverted-file rebuild, for gfx950.
//
// The object set's term-major view (entries ordered by (term, object), built
// once) is stably radix-sorted by the entries' current cluster, which leaves
// every cluster's entries grouped by term: each run of equal (cluster, term)
// is one nonzero of the new mean.  Its member sum is accumulated in integer
// fixed point with a per-term scale that holds every FP32 value of the term
// exactly, so the sum is the exact real sum (independent of order and thread
// count: a deterministic segmented reduction).  The mean is then the sum
// divided by |C_j| and by the FP64 2-norm, as the paper orders the update.
// Clusters without members keep their previous mean.
#include "ivf_internal.h"
#include "kernels.h"
#include "update.h"

namespace ivf {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int per_thread = 1) {
    int64_t b = (n + (int64_t)kThreads * per_thread - 1) / ((int64_t)kThreads * per_thread);
    return (unsigned)(b > 0 ? b : 1);
}

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

// Largest value (as double bits: non-negative doubles order like their bit
// patterns) and longest row of a wave's rows, one atomic each per wave.
__device__ inline void wave_max_out(double vmax, int64_t len, Counters* cnt) {
    unsigned long long vb = (unsigned long long)__double_as_longlong(vmax);
    unsigned long long lb = (unsigned long long)len;
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        const unsigned long long ov = (unsigned long long)__shfl_xor((long long)vb, o, kWave);
        const unsigned long long ol = (unsigned long long)__shfl_xor((long long)lb, o, kWave);
        vb = ov > vb ? ov : vb;
        lb = ol > lb ? ol : lb;
    }
    if (lane_id() == 0) {
        if (vb) atomicMax(&cnt->vmax_bits, vb);
        if (lb) atomicMax(&cnt->nmax, lb);
    }
}

__global__ void k_validate_objects(ObjectView x, Counters* cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (x.x_ptr[0] != 0 || x.x_ptr[x.n] != x.nnz))
        atomicOr(&cnt->error_flags, (unsigned long long)kBadPtr);
    unsigned f = 0;
    double vmax = 0.0;
    int64_t len = 0;
    if (i < x.n) {
        const int64_t a = x.x_ptr[i], b = x.x_ptr[i + 1];
        if (a < 0 || b < a || b > x.nnz) {
            f = kBadPtr;
        } else {
            len = b - a;
            int32_t prevt = -1;
            for (int64_t e = a; e < b; ++e) {
                const int32_t t = x.x_idx[e];
                const float v = x.x_val[e];
                if (t < 0 || t >= x.d) f |= kBadIndex;
                else if (t <= prevt) f |= kBadOrder;
                prevt = t;
                if (!isfinite(v)) f |= kNonFinite;
                else if (!(v > 0.f)) f |= kNonPositive;
                else vmax = fmax(vmax, (double)v);
            }
        }
    }
    if (f) atomicOr(&cnt->error_flags, (unsigned long long)f);
    wave_max_out(vmax, len, cnt);
}

__global__ void k_validate_means(const int64_t* ptr, const int32_t* idx, const double* val,
                                 int32_t k, int64_t d, int64_t nnz, Counters* cnt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0 && (ptr[0] != 0 || ptr[k] != nnz))
        atomicOr(&cnt->error_flags, (unsigned long long)kBadPtr);
    unsigned f = 0;
    double vmax = 0.0;
    int64_t len = 0;
    if (j < k) {
        const int64_t a = ptr[j], b = ptr[j + 1];
        if (a < 0 || b < a || b > nnz) {
            f = kBadPtr;
        } else {
            len = b - a;
            int32_t prevt = -1;
            for (int64_t e = a; e < b; ++e) {
                const int32_t t = idx[e];
                const double v = val[e];
                if (t < 0 || t >= d) f |= kBadIndex;
                else if (t <= prevt) f |= kBadOrder;
                prevt = t;
                if (!isfinite(v)) f |= kNonFinite;
                else if (!(v > 0.0)) f |= kNonPositive;
                else vmax = fmax(vmax, v);
            }
        }
    }
    if (f) atomicOr(&cnt->error_flags, (unsigned long long)f);
    wave_max_out(vmax, len, cnt);
}

__global__ void k_row_ids(const int64_t* ptr, int64_t n, int32_t* rowid) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) rowid[e] = (int32_t)i;
}

__global__ void k_iota(uint32_t* out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)i;
}

__global__ void k_copy_keys(const int32_t* in, uint32_t* out, int64_t n,
                            const int64_t* n_dev = nullptr) {
    n = bounded_count(n, n_dev);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)in[i];
}

__global__ void k_build_xt(const uint32_t* st, const uint32_t* sp, const int32_t* rowid,
                           const float* x_val, int64_t nnz, int32_t* xt_obj, uint2* xt_tv) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = sp[q];
        xt_obj[q] = rowid[e];
        xt_tv[q] = make_uint2(st[q], __float_as_uint(x_val[e]));
    }
}

__global__ void k_term_init(int32_t* emin, int32_t* emax, int32_t* count, int64_t d) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d) return;
    emin[t] = 1 << 30;
    emax[t] = -(1 << 30);
    count[t] = 0;
}

__global__ void k_term_stats(const int32_t* x_idx, const float* x_val, int64_t nnz,
                             int32_t* emin, int32_t* emax, int32_t* count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t t = x_idx[e];
        int32_t eb = (int32_t)((__float_as_uint(x_val[e]) >> 23) & 0xffu);
        if (eb == 0) eb = 1;   // subnormals share the smallest normal exponent's lsb
        atomicMin(&emin[t], eb);
        atomicMax(&emax[t], eb);
        atomicAdd(&count[t], 1);
    }
}

__global__ void k_term_shift(const int32_t* emin, const int32_t* emax, const int32_t* count,
                             int64_t d, int16_t* shift, Counters* cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d) return;
    const int32_t c = count[t];
    if (c == 0) {
        shift[t] = 0;
        return;
    }
    // lsb of the smallest value: every value of the term is an integer multiple
    const int32_t s_exact = (emin[t] - 127) - 23;
    const int32_t logc = c > 1 ? 32 - __clz((unsigned)(c - 1)) : 0;
    // any member sum < c * 2^(emax + 1); keep it below 2^63 in lsb units
    const int32_t need = logc + (emax[t] - 127 + 1) - s_exact;
    int32_t s = s_exact;
    if (need > 62) {
        s += need - 62;
        atomicAdd(&cnt->inexact, 1ull);   // terms whose sums are rounded
    }
    shift[t] = (int16_t)s;
}

// ----------------------------------------------------------------- update
__global__ void k_keys(const int32_t* __restrict__ xt_obj, const int32_t* __restrict__ assign,
                       int64_t nnz, int32_t k, uint32_t* __restrict__ keys) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = assign[xt_obj[q]];
        keys[q] = (a >= 0 && a < k) ? (uint32_t)a : (uint32_t)k;
    }
}

__global__ void k_sizes(const int32_t* __restrict__ assign, int64_t n, int32_t k,
                        int64_t* __restrict__ size) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = assign[i];
        if (a >= 0 && a < k)
            atomicAdd(reinterpret_cast<unsigned long long*>(&size[a]), 1ull);
    }
}

__global__ void k_zero_i64(int64_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Entries sorted by cluster carry their (term, value) payload, so runs of
// equal (cluster, term) are found by reading neighbours, not by gathers.
// tmask: the bits of the payload's first word that hold the term (the others
// mark a delta entry that subtracts its value, see k_delta_emit).
__global__ void k_seg_flags(const uint32_t* __restrict__ keys, const uint2* __restrict__ pay,
                            int64_t nnz, int32_t k, uint32_t tmask, uint32_t* __restrict__ flag,
                            int64_t* scal) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t key = keys[q];
        const bool valid = key < (uint32_t)k;
        uint32_t f = 0;
        if (valid) {
            if (q == 0) f = 1;
            else {
                const uint32_t kp = keys[q - 1];
                f = (kp != key || ((pay[q].x ^ pay[q - 1].x) & tmask) != 0u) ? 1u : 0u;
            }
            if (q == nnz - 1 || keys[q + 1] >= (uint32_t)k) scal[0] = q + 1;
        }
        flag[q] = f;
    }
}

__global__ void k_seg_count(const uint32_t* flag, const uint32_t* segpos, int64_t nnz,
                            int64_t* scal) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        scal[1] = nnz > 0 ? (int64_t)segpos[nnz - 1] + flag[nnz - 1] : 0;
}

__global__ void k_zero_segs(unsigned long long* acc, const int64_t* scal, int64_t cap) {
    const int64_t ns = scal[1];
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < ns && s < cap;
         s += (int64_t)gridDim.x * blockDim.x)
        acc[s] = 0ull;
}

__device__ inline unsigned long long to_fixed(float v, int sh) {
    // exact when the term's scale holds v (the common case), else rounded to nearest
    return (unsigned long long)llrint(ldexp((double)v, -sh));
}

constexpr int kRun = 8;

__device__ inline unsigned long long shfl_up_u64(unsigned long long x, int d) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, kWave);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, kWave);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ inline int64_t shfl_up_i64(int64_t x, int d) {
    return (int64_t)shfl_up_u64((unsigned long long)x, d);
}
__device__ inline int64_t shfl_down_i64(int64_t x, int d) {
    const uint32_t lo = (uint32_t)__shfl_down((int)(uint32_t)x, d, kWave);
    const uint32_t hi = (uint32_t)__shfl_down((int)(uint32_t)(x >> 32), d, kWave);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline int64_t readlane_i64(int64_t x, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Fixed-point sums of the (cluster, term) segments.  One wave takes 64 * kRun
// consecutive entries (in cluster order) as kRun chunks of 64; within a chunk
// an inclusive segmented scan over the lanes (segments are contiguous) sums
// each run, and the lane that ends a run adds it to the segment's
// accumulator.  A run reaching the chunk's last lane is carried into the next
// chunk, so a long segment costs one atomic per wave, not one per lane.  The
// sums are integers: exact and independent of the order of the additions.
// Entries whose payload carries bits outside tmask subtract their value (two's
// complement: the sums are exact modulo 2^64, and every final sum is in range).
__global__ __launch_bounds__(kThreads) void k_seg_sums(const uint32_t* __restrict__ keys,
                                                       const uint2* __restrict__ pay,
                                                       uint32_t tmask,
                                                       const uint32_t* __restrict__ flag,
                                                       const uint32_t* __restrict__ segpos,
                                                       const int16_t* __restrict__ shift,
                                                       const int64_t* scal,
                                                       unsigned long long* __restrict__ acc,
                                                       int32_t* __restrict__ seg_j,
                                                       int32_t* __restrict__ seg_t) {
    const int64_t nv = scal[0];
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t qbase = wave * ((int64_t)kWave * kRun);
    if (qbase >= nv) return;   // the same for all lanes of the wave
    int64_t carry_seg = -1;    // wave-uniform
    unsigned long long carry = 0;
    for (int u = 0; u < kRun; ++u) {
        const int64_t q = qbase + (int64_t)u * kWave + lane;
        const bool valid = q < nv;
        int64_t sg = -1;
        unsigned long long v = 0;
        if (valid) {
            const uint2 tv = pay[q];
            const int32_t t = (int32_t)(tv.x & tmask);
            sg = (int64_t)segpos[q] + flag[q] - 1;
            if (flag[q]) {
                seg_j[sg] = (int32_t)keys[q];
                seg_t[sg] = t;
            }
            v = to_fixed(__uint_as_float(tv.y), shift[t]);
            if (tv.x & ~tmask) v = 0ull - v;
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const unsigned long long ov = shfl_up_u64(v, d);
            const int64_t os = shfl_up_i64(sg, d);
            if (lane >= d && os == sg) v += ov;
        }
        const int64_t first = readlane_i64(sg, 0);
        if (carry_seg >= 0 && first != carry_seg) {   // the carried run ended with the last chunk
            if (lane == 0) atomicAdd(&acc[carry_seg], carry);
            carry_seg = -1;
            carry = 0;
        }
        if (carry_seg >= 0 && sg == carry_seg) v += carry;
        const int64_t next = shfl_down_i64(sg, 1);
        if (valid && lane < kWave - 1 && next != sg) atomicAdd(&acc[sg], v);
        const int64_t last = readlane_i64(sg, kWave - 1);
        if (last >= 0) {   // the last lane's run may continue into the next chunk
            carry_seg = last;
            carry = (unsigned long long)readlane_i64((int64_t)v, kWave - 1);
        } else {
            carry_seg = -1;
            carry = 0;
        }
    }
    if (carry_seg >= 0 && lane == 0) atomicAdd(&acc[carry_seg], carry);
}

__device__ inline int64_t lower_bound_i32(const int32_t* a, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void k_cstart(const int32_t* seg_j, const int64_t* scal, int32_t k, int64_t* cstart) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > k) return;
    cstart[j] = lower_bound_i32(seg_j, 0, scal[1], (int32_t)j);
}

__device__ inline double seg_value(const unsigned long long* acc, const int32_t* seg_t,
                                   const int16_t* shift, int64_t s) {
    return ldexp((double)acc[s], (int)shift[seg_t[s]]);
}

// The norm pass works on fixed chunks of kNormChunk segments, so its
// parallelism does not depend on k (a few huge clusters or many small ones).
// Work items per cluster: ceil(segments / kNormChunk) for a cluster with members.
__global__ void k_norm_items(const int64_t* __restrict__ size, const int64_t* __restrict__ cstart,
                             int32_t k, int64_t* __restrict__ items) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > k) return;
    if (j == k) {
        items[k] = 0;
        return;
    }
    const int64_t len = cstart[j + 1] - cstart[j];
    items[j] = size[j] > 0 ? (len + kNormChunk - 1) / kNormChunk : 0;
}

// First place p in [lo, hi) with a[p] >= x (hi when there is none), a sorted
// a, searched from the guess g: steps of doubling length away from g bracket
// the place, which bisection then finds.  A guess off by m costs about
// 2 log2(m) reads, one when it is right.
__device__ inline int64_t seek_i32(const int32_t* a, int64_t lo, int64_t hi, int64_t g,
                                   int32_t x) {
    g = g < lo ? lo : (g > hi ? hi : g);
    int64_t l, r;   // the place lies in [l, r]
    if (g < hi) {
        const int32_t v = a[g];
        if (v == x) return g;
        if (v < x) {   // above g
            l = g + 1;
            r = hi;
            for (int64_t step = 1;; step <<= 1) {
                const int64_t q = g + step;
                if (q >= hi) break;
                if (a[q] >= x) { r = q; break; }
                l = q + 1;
            }
            return lower_bound_i32(a, l, r, x);
        }
    }
    // a[g] > x, or g == hi: at or below g
    l = lo;
    r = g;
    for (int64_t step = 1;; step <<= 1) {
        const int64_t q = g - step;
        if (q < lo) break;
        if (a[q] < x) { l = q + 1; break; }
        r = q;
    }
    return lower_bound_i32(a, l, r, x);
}

// One wave per work item (the scanned item offsets locate its cluster):
// partial FP64 sums over one chunk of the cluster's segments of w^2, with
// w = s / |C_j|, and of mu_j(old) . s (the exact objective's share).
// Lane-strided partials and a fixed butterfly: deterministic.  The old row
// differs little from the new one, so each term is sought from the place the
// previous step's last term had, moved by the distance between the two.
__global__ __launch_bounds__(kThreads) void k_norm_parts(UpdateArgs a) {
    const int64_t it = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = lane_id();
    if (it >= a.norm_items[a.k]) return;
    int64_t lo = 0, hi = a.k;   // last cluster j with norm_items[j] <= it
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.norm_items[mid] <= it) lo = mid; else hi = mid;
    }
    const int64_t j = lo;
    const int64_t c = it - a.norm_items[j];
    const int64_t s0 = a.cstart[j] + c * kNormChunk;
    const int64_t s1 = min(a.cstart[j + 1], s0 + kNormChunk);
    const int64_t ob = a.old_ptr[j], oe = a.old_ptr[j + 1];
    const double dn = (double)a.size[j];
    double ss = 0.0, op = 0.0;
    int64_t from = ob;                 // wave-uniform: no term of this step lies before it
    int64_t off = ob - a.cstart[j];    // wave-uniform: old place minus new place, guessed
    for (int64_t base = s0; base < s1; base += kWave) {   // wave-uniform trip count
        const int64_t s = base + lane;
        int64_t p = from;
        if (s < s1) {
            const double sv = seg_value(a.seg_acc, a.seg_t, a.shift, s);
            const double w = sv / dn;
            ss += w * w;
            const int32_t t = a.seg_t[s];
            p = seek_i32(a.old_idx, from, oe, s + off, t);
            if (p < oe && a.old_idx[p] == t) op += a.old_val[p] * sv;
        }
        const int last = s1 - 1 - base < kWave - 1 ? (int)(s1 - 1 - base) : kWave - 1;
        from = readlane_i64(p, last);
        off = from - (base + last);
    }
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        ss += __shfl_xor(ss, o, kWave);
        op += __shfl_xor(op, o, kWave);
    }
    if (lane == 0) {
        a.norm_part[2 * it] = ss;
        a.norm_part[2 * it + 1] = op;
    }
}

// One thread per cluster: its items' partials summed in item order, the FP64
// norm, the objective share and the new row length; a cluster without
// members keeps its row.
__global__ void k_norm_final(UpdateArgs a) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.k) return;
    if (a.size[j] == 0) {
        a.newcnt[j] = a.old_ptr[j + 1] - a.old_ptr[j];
        a.nrm[j] = 0.0;
        a.objpart[j] = 0.0;
        atomicAdd(&a.cnt->empty, 1ull);
        return;
    }
    double ss = 0.0, op = 0.0;
    for (int64_t i = a.norm_items[j]; i < a.norm_items[j + 1]; ++i) {
        ss += a.norm_part[2 * i];
        op += a.norm_part[2 * i + 1];
    }
    a.nrm[j] = sqrt(ss);
    a.objpart[j] = op;
    a.newcnt[j] = a.cstart[j + 1] - a.cstart[j];
}

// The new rows.  Waves below norm_items[k] take one work item each (a chunk
// of kNormChunk segments of a cluster with members, as in the norm pass, so
// one huge cluster does not hold up the launch); wave item_cap + j copies the
// old row of cluster j when it has no members.
__global__ __launch_bounds__(kThreads) void k_fill(UpdateArgs a, int64_t item_cap) {
    const int64_t it = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = lane_id();
    if (a.new_ptr[a.k] > a.new_cap) {   // the new means do not fit: flag, write nothing
        if (it == 0 && lane == 0) atomicOr(&a.cnt->error_flags, (unsigned long long)kOverflow);
        return;
    }
    if (it >= item_cap) {
        const int64_t j = it - item_cap;
        if (j >= a.k || a.size[j] != 0) return;
        const int64_t p0 = a.new_ptr[j];
        const int64_t ob = a.old_ptr[j], oe = a.old_ptr[j + 1];
        for (int64_t e = ob + lane; e < oe; e += kWave) {
            a.new_idx[p0 + (e - ob)] = a.old_idx[e];
            a.new_val[p0 + (e - ob)] = a.old_val[e];
            a.new_row[p0 + (e - ob)] = (int32_t)j;
        }
        return;
    }
    if (it >= a.norm_items[a.k]) return;
    int64_t lo = 0, hi = a.k;   // last cluster j with norm_items[j] <= it
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.norm_items[mid] <= it) lo = mid; else hi = mid;
    }
    const int64_t j = lo;
    const int64_t row0 = a.cstart[j];
    const int64_t s0 = row0 + (it - a.norm_items[j]) * kNormChunk;
    const int64_t s1 = min(a.cstart[j + 1], s0 + kNormChunk);
    const int64_t p0 = a.new_ptr[j];
    const double dn = (double)a.size[j], nr = a.nrm[j];
    for (int64_t s = s0 + lane; s < s1; s += kWave) {
        const double w = seg_value(a.seg_acc, a.seg_t, a.shift, s) / dn;
        a.new_idx[p0 + (s - row0)] = a.seg_t[s];
        a.new_val[p0 + (s - row0)] = w / nr;
        a.new_row[p0 + (s - row0)] = (int32_t)j;
    }
}

__global__ __launch_bounds__(kThreads) void k_sum_k(const double* part, int32_t k, double* out) {
    __shared__ double sh[kThreads];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < k; i += kThreads) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_mean_rows(const int64_t* ptr, int32_t k, int32_t* row) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) row[e] = (int32_t)j;
}

// ------------------------------------------------------ incremental update
// The member sums of every (cluster, term) are exact integers, so the sums of
// a new assignment are the stored sums of the previous one, minus the values
// of the objects that left each cluster, plus those of the objects that
// joined it: bit for bit what the full segmented reduction gives.  The stored
// table lists (cluster, term, sum) for every nonzero sum in (cluster, term)
// order.

__device__ inline int32_t valid_cluster(int32_t a, int32_t k) { return (a >= 0 && a < k) ? a : -1; }

// Delta entries of object i: its row once for the cluster it left and once
// for the cluster it joined (0 if unchanged).  cnt[n] = 0 for the scan.
__global__ void k_delta_count(const int64_t* __restrict__ x_ptr, int64_t n,
                              const int32_t* __restrict__ assign,
                              const int32_t* __restrict__ old_assign, int32_t k,
                              int64_t* __restrict__ cnt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0;
        if (i < n) {
            const int32_t a = valid_cluster(assign[i], k), o = valid_cluster(old_assign[i], k);
            if (a != o) c = (x_ptr[i + 1] - x_ptr[i]) * ((a >= 0) + (o >= 0));
        }
        cnt[i] = c;
    }
}

// Cluster sizes of `assign` from those of `old_assign`: each changed object
// leaves its old cluster and joins its new one.
__global__ void k_delta_sizes(const int32_t* __restrict__ assign,
                              const int32_t* __restrict__ old_assign, int64_t n, int32_t k,
                              int64_t* __restrict__ size) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = valid_cluster(assign[i], k), o = valid_cluster(old_assign[i], k);
        if (a == o) continue;
        if (o >= 0) atomicAdd(reinterpret_cast<unsigned long long*>(&size[o]), ~0ull);   // -1
        if (a >= 0) atomicAdd(reinterpret_cast<unsigned long long*>(&size[a]), 1ull);
    }
}

// The delta entries of the changed objects at their scanned offsets, keyed by
// term: payload (cluster | 2^31 if the entry subtracts, FP32 value bits).  A
// wave takes 64 consecutive objects and copies the rows of the changed ones
// one after the other, its lanes reading and writing consecutive entries.
__global__ void k_delta_emit(const int64_t* __restrict__ x_ptr, const int32_t* __restrict__ x_idx,
                             const float* __restrict__ x_val, int64_t n,
                             const int32_t* __restrict__ assign,
                             const int32_t* __restrict__ old_assign, int32_t k,
                             const int64_t* __restrict__ off, uint32_t* __restrict__ keys,
                             uint2* __restrict__ pay) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;   // objects per sweep of the grid
    for (int64_t g0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane; g0 < n;
         g0 += stride) {   // wave-uniform
        const int64_t i = g0 + lane;
        uint64_t changed = __ballot(i < n && off[i + 1] != off[i]);
        while (changed) {
            const int64_t obj = g0 + (__ffsll((unsigned long long)changed) - 1);
            changed &= changed - 1;
            const int32_t a = valid_cluster(assign[obj], k), o = valid_cluster(old_assign[obj], k);
            const int64_t hb = x_ptr[obj], len = x_ptr[obj + 1] - hb;
            const int64_t q = off[obj];
            const int64_t qa = q + (o >= 0 ? len : 0);   // the added copy follows the subtracted one
            for (int64_t e = lane; e < len; e += kWave) {
                const uint32_t t = (uint32_t)x_idx[hb + e];
                const uint32_t v = __float_as_uint(x_val[hb + e]);
                if (o >= 0) {
                    keys[q + e] = t;
                    pay[q + e] = make_uint2((uint32_t)o | 0x80000000u, v);
                }
                if (a >= 0) {
                    keys[qa + e] = t;
                    pay[qa + e] = make_uint2((uint32_t)a, v);
                }
            }
        }
    }
}

// Sorted by term, the entries are keyed again by cluster (the payload then
// carries the term and the sign bit); a stable sort by cluster follows.
__global__ void k_delta_rekey(uint32_t* __restrict__ keys, uint2* __restrict__ pay, int64_t m) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = keys[q];
        const uint2 p = pay[q];
        keys[q] = p.x & 0x7fffffffu;
        pay[q] = make_uint2(t | (p.x & 0x80000000u), p.y);
    }
}

// Each delta segment (cluster j, term t, signed sum) added into the table if
// (j, t) is there (cstart: the table's cluster starts); otherwise it is an
// insertion before table position lb (its sum is then a positive total of
// joined values), counted in add[lb].  ins[d] = 1 marks an insertion; it is
// cleared up to `cap` (>= the segment count), the length the host scans.
__global__ void k_delta_apply(const int32_t* __restrict__ dj, const int32_t* __restrict__ dt,
                              const unsigned long long* __restrict__ dacc,
                              const int64_t* __restrict__ scal, int64_t cap,
                              const int64_t* __restrict__ cstart,
                              const int32_t* __restrict__ tab_t,
                              unsigned long long* __restrict__ tab_acc,
                              uint32_t* __restrict__ ins, uint32_t* __restrict__ ins_lb,
                              uint32_t* __restrict__ add) {
    const int64_t nd = scal[1];
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < cap;
         d += (int64_t)gridDim.x * blockDim.x) {
        if (d >= nd) {
            ins[d] = 0;
            continue;
        }
        const int32_t j = dj[d], t = dt[d];
        const int64_t e = cstart[j + 1];
        int64_t lo = cstart[j], hi = e;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (tab_t[mid] < t) lo = mid + 1; else hi = mid;
        }
        const unsigned long long v = dacc[d];
        uint32_t f = 0;
        if (lo < e && tab_t[lo] == t) {
            tab_acc[lo] += v;   // one delta segment per (j, t): no other writer
        } else if (v != 0ull) {
            f = 1;
            ins_lb[d] = (uint32_t)lo;
            atomicAdd(&add[lo], 1u);
        }
        ins[d] = f;
    }
}

// Per table position p (and p = m for insertions after the last entry): the
// entry survives if its sum is nonzero (high word) and add[p] insertions go
// before it (low word); one scan of the packed counts gives both prefixes.
__global__ void k_merge_counts(const unsigned long long* __restrict__ tab_acc, int64_t m,
                               const uint32_t* __restrict__ add, int64_t* __restrict__ c) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= m;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t keep = (p < m && tab_acc[p] != 0ull) ? 1 : 0;
        c[p] = (keep << 32) | (int64_t)add[p];
    }
}

// The new table: surviving entries after the insertions that precede them,
// insertions at the surviving entries before their position plus their rank
// among all insertions.  The new entry count goes to scal[1].
__global__ void k_merge_scatter(const int32_t* __restrict__ tab_j, const int32_t* __restrict__ tab_t,
                                const unsigned long long* __restrict__ tab_acc, int64_t m,
                                const uint32_t* __restrict__ add, const int64_t* __restrict__ cs,
                                const int32_t* __restrict__ dj, const int32_t* __restrict__ dt,
                                const unsigned long long* __restrict__ dacc,
                                const uint32_t* __restrict__ ins, const uint32_t* __restrict__ ins_lb,
                                const uint32_t* __restrict__ ipos, int64_t* __restrict__ scal,
                                int32_t* __restrict__ nj, int32_t* __restrict__ nt,
                                unsigned long long* __restrict__ nacc) {
    const int64_t nd = scal[1];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t p = g; p < m; p += stride) {
        const unsigned long long v = tab_acc[p];
        if (v == 0ull) continue;
        const int64_t at = (cs[p] >> 32) + (cs[p] & 0xffffffffll) + add[p];
        nj[at] = tab_j[p];
        nt[at] = tab_t[p];
        nacc[at] = v;
    }
    for (int64_t d = g; d < nd; d += stride) {
        if (!ins[d]) continue;
        const int64_t at = (cs[ins_lb[d]] >> 32) + ipos[d];
        nj[at] = dj[d];
        nt[at] = dt[d];
        nacc[at] = dacc[d];
    }
}

__global__ void k_merge_total(const int64_t* __restrict__ cs, const uint32_t* __restrict__ add,
                              int64_t m, int64_t* __restrict__ scal) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        scal[1] = (cs[m] >> 32) + (cs[m] & 0xffffffffll) + add[m];
}

// The full reduction's segments become the stored table (count at scal[1]).
__global__ void k_copy_table(const int32_t* __restrict__ sj, const int32_t* __restrict__ st,
                             const unsigned long long* __restrict__ sacc,
                             const int64_t* __restrict__ scal, int64_t cap,
                             int32_t* __restrict__ tj, int32_t* __restrict__ tt,
                             unsigned long long* __restrict__ tacc) {
    const int64_t m = min(scal[1], cap);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * blockDim.x) {
        tj[p] = sj[p];
        tt[p] = st[p];
        tacc[p] = sacc[p];
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_scatter_seeds(const int32_t* seeds, int32_t k, int64_t n, int32_t* assign) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    const int32_t i = seeds[j];
    if (i >= 0 && i < n) assign[i] = (int32_t)j;
}

inline int bits_for(int64_t maxval) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) <= maxval) ++b;
    return b;
}

inline unsigned capped(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

#define HIP_RET(x)                           \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

}  // namespace

hipError_t launch_validate_objects(const ObjectView& x, Counters* cnt, hipStream_t s) {
    k_validate_objects<<<grid_for(x.n + 1), kThreads, 0, s>>>(x, cnt);
    return hipGetLastError();
}

hipError_t launch_validate_means(const int64_t* ptr, const int32_t* idx, const double* val,
                                 int32_t k, int64_t d, int64_t nnz, Counters* cnt,
                                 hipStream_t s) {
    k_validate_means<<<grid_for(k + 1), kThreads, 0, s>>>(ptr, idx, val, k, d, nnz, cnt);
    return hipGetLastError();
}

hipError_t launch_row_ids(const int64_t* ptr, int64_t n, int32_t* rowid, hipStream_t s) {
    k_row_ids<<<grid_for(n), kThreads, 0, s>>>(ptr, n, rowid);
    return hipGetLastError();
}

hipError_t launch_iota(uint32_t* out, int64_t n, hipStream_t s) {
    k_iota<<<capped(n), kThreads, 0, s>>>(out, n);
    return hipGetLastError();
}

hipError_t launch_copy_keys(const int32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
    k_copy_keys<<<capped(n), kThreads, 0, s>>>(in, out, n);
    return hipGetLastError();
}

hipError_t launch_build_xt(const uint32_t* st, const uint32_t* sp, const int32_t* rowid,
                           const float* x_val, int64_t nnz, int32_t* xt_obj, uint2* xt_tv,
                           hipStream_t s) {
    k_build_xt<<<capped(nnz), kThreads, 0, s>>>(st, sp, rowid, x_val, nnz, xt_obj, xt_tv);
    return hipGetLastError();
}

hipError_t launch_term_shift(const int32_t* x_idx, const float* x_val, int64_t nnz, int64_t d,
                             int32_t* emin, int32_t* emax, int32_t* count, int16_t* shift,
                             Counters* cnt, hipStream_t s) {
    k_term_init<<<grid_for(d), kThreads, 0, s>>>(emin, emax, count, d);
    k_term_stats<<<capped(nnz), kThreads, 0, s>>>(x_idx, x_val, nnz, emin, emax, count);
    k_term_shift<<<grid_for(d), kThreads, 0, s>>>(emin, emax, count, d, shift, cnt);
    return hipGetLastError();
}

namespace {
hipError_t launch_sizes(const int32_t* assign, int64_t n, int32_t k, int64_t* size, int64_t* scal,
                        hipStream_t s) {
    k_zero_i64<<<capped(k + 1), kThreads, 0, s>>>(size, k);
    k_zero_i64<<<1, kThreads, 0, s>>>(scal, 4);
    k_sizes<<<capped(n), kThreads, 0, s>>>(assign, n, k, size);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_update_sums(UpdateArgs& a, hipStream_t s) {
    HIP_RET(launch_update_segments(a, s));
    return launch_update_norms(a, s);
}

hipError_t launch_update_segments(UpdateArgs& a, hipStream_t s) {
    const int64_t nnz = a.nnz;
    HIP_RET(launch_sizes(a.assign, a.n, a.k, a.size, a.scal, s));
    if (nnz > 0) {
        k_keys<<<capped(nnz), kThreads, 0, s>>>(a.xt_obj, a.assign, nnz, a.k, a.keys);
        HIP_RET(hipGetLastError());
        // stable sort by cluster; the (term, value) payload moves with its key.
        // The segment-sum buffer (8 B per entry, written only after the sort)
        // is the payload's second buffer.
        HIP_RET(radix_sort_pairs_u64(a.keys, a.pay, a.keys_alt,
                                     reinterpret_cast<uint2*>(a.seg_acc), nnz, bits_for(a.k),
                                     a.tmp, s, a.xt_tv));
        k_seg_flags<<<capped(nnz), kThreads, 0, s>>>(a.keys, a.pay, nnz, a.k, 0xffffffffu, a.flag,
                                                     a.scal);
        HIP_RET(hipGetLastError());
        HIP_RET(exclusive_scan_u32(a.flag, a.segpos, nnz, a.tmp, s));
        k_seg_count<<<1, 64, 0, s>>>(a.flag, a.segpos, nnz, a.scal);
        k_zero_segs<<<capped(nnz), kThreads, 0, s>>>(a.seg_acc, a.scal, nnz);
        k_seg_sums<<<grid_for(nnz, kRun), kThreads, 0, s>>>(a.keys, a.pay, 0xffffffffu, a.flag,
                                                            a.segpos, a.shift, a.scal, a.seg_acc,
                                                            a.seg_j, a.seg_t);
        HIP_RET(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t launch_update_norms(UpdateArgs& a, hipStream_t s) {
    k_cstart<<<grid_for(a.k + 1), kThreads, 0, s>>>(a.seg_j, a.scal, a.k, a.cstart);
    k_norm_items<<<grid_for(a.k + 1), kThreads, 0, s>>>(a.size, a.cstart, a.k, a.norm_items);
    HIP_RET(hipGetLastError());
    HIP_RET(exclusive_scan_i64(a.norm_items, a.norm_items, (int64_t)a.k + 1, a.tmp, s));
    // one wave per item; the item count is bounded by k + nnz / kNormChunk + 1
    k_norm_parts<<<grid_for(norm_item_bound(a.k, a.nnz) * kWave), kThreads, 0, s>>>(a);
    k_norm_final<<<grid_for(a.k), kThreads, 0, s>>>(a);
    HIP_RET(hipGetLastError());
    // new row pointers: exclusive scan of k + 1 counts (the last is 0)
    k_zero_i64<<<1, 64, 0, s>>>(a.newcnt + a.k, 1);
    HIP_RET(exclusive_scan_i64(a.newcnt, a.new_ptr, (int64_t)a.k + 1, a.tmp, s));
    return hipGetLastError();
}

hipError_t launch_delta_count(const int64_t* x_ptr, int64_t n, const int32_t* assign,
                              const int32_t* old_assign, int32_t k, int64_t* off, void* tmp,
                              hipStream_t s) {
    k_delta_count<<<capped(n + 1), kThreads, 0, s>>>(x_ptr, n, assign, old_assign, k, off);
    HIP_RET(hipGetLastError());
    return exclusive_scan_i64(off, off, n + 1, tmp, s);
}

hipError_t launch_delta_update(DeltaArgs& a, hipStream_t s) {
    // a.size holds the sizes of a.old_assign (the last update's assignment)
    k_zero_i64<<<1, kThreads, 0, s>>>(a.scal, 4);
    k_delta_sizes<<<capped(a.n), kThreads, 0, s>>>(a.assign, a.old_assign, a.n, a.k, a.size);
    HIP_RET(hipGetLastError());
    const int64_t m = a.entries;
    if (m > 0) {
        k_delta_emit<<<capped(a.n), kThreads, 0, s>>>(a.x_ptr, a.x_idx, a.x_val, a.n, a.assign,
                                                      a.old_assign, a.k, a.off, a.keys, a.pay);
        HIP_RET(hipGetLastError());
        // (cluster, term) order: stable by term, then stable by cluster
        HIP_RET(radix_sort_pairs_u64(a.keys, a.pay, a.keys_alt, a.pay_alt, m,
                                     bits_for(a.d - 1 > 0 ? a.d - 1 : 1), a.tmp, s, nullptr));
        k_delta_rekey<<<capped(m), kThreads, 0, s>>>(a.keys, a.pay, m);
        HIP_RET(hipGetLastError());
        HIP_RET(radix_sort_pairs_u64(a.keys, a.pay, a.keys_alt, a.pay_alt, m, bits_for(a.k),
                                     a.tmp, s, nullptr));
        k_seg_flags<<<capped(m), kThreads, 0, s>>>(a.keys, a.pay, m, a.k, 0x7fffffffu, a.flag,
                                                   a.scal);
        HIP_RET(hipGetLastError());
        HIP_RET(exclusive_scan_u32(a.flag, a.segpos, m, a.tmp, s));
        k_seg_count<<<1, 64, 0, s>>>(a.flag, a.segpos, m, a.scal);
        k_zero_segs<<<capped(m), kThreads, 0, s>>>(a.dacc, a.scal, m);
        k_seg_sums<<<grid_for(m, kRun), kThreads, 0, s>>>(a.keys, a.pay, 0x7fffffffu, a.flag,
                                                          a.segpos, a.shift, a.scal, a.dacc,
                                                          a.dj, a.dt);
        HIP_RET(hipGetLastError());
    }
    // merge the delta segments (count at scal[1]) into the table
    const int64_t tn = a.tab_n;
    k_fill_i32<<<capped(tn + 1), kThreads, 0, s>>>(reinterpret_cast<int32_t*>(a.add), tn + 1, 0);
    if (m > 0) {
        k_delta_apply<<<capped(m), kThreads, 0, s>>>(a.dj, a.dt, a.dacc, a.scal, m, a.cstart,
                                                     a.tab_t, a.tab_acc, a.ins, a.ins_lb, a.add);
        HIP_RET(hipGetLastError());
        HIP_RET(exclusive_scan_u32(a.ins, a.ipos, m, a.tmp, s));
    }
    k_merge_counts<<<capped(tn + 1), kThreads, 0, s>>>(a.tab_acc, tn, a.add, a.cs);
    HIP_RET(hipGetLastError());
    HIP_RET(exclusive_scan_i64(a.cs, a.cs, tn + 1, a.tmp, s));
    k_merge_scatter<<<capped(std::max<int64_t>(tn, m)), kThreads, 0, s>>>(
        a.tab_j, a.tab_t, a.tab_acc, tn, a.add, a.cs, a.dj, a.dt, a.dacc, a.ins, a.ins_lb, a.ipos,
        a.scal, a.new_j, a.new_t, a.new_acc);
    k_merge_total<<<1, 64, 0, s>>>(a.cs, a.add, tn, a.scal);
    return hipGetLastError();
}

hipError_t launch_copy_table(const int32_t* sj, const int32_t* st, const unsigned long long* sacc,
                             const int64_t* scal, int64_t cap, int32_t* tj, int32_t* tt,
                             unsigned long long* tacc, hipStream_t s) {
    k_copy_table<<<capped(cap), kThreads, 0, s>>>(sj, st, sacc, scal, cap, tj, tt, tacc);
    return hipGetLastError();
}

hipError_t launch_update_fill(UpdateArgs& a, hipStream_t s) {
    const int64_t items = norm_item_bound(a.k, a.nnz);
    k_fill<<<grid_for((items + a.k) * kWave), kThreads, 0, s>>>(a, items);
    return hipGetLastError();
}

hipError_t launch_objective_exact(const double* objpart, int32_t k, double* out,
                                  hipStream_t s) {
    k_sum_k<<<1, kThreads, 0, s>>>(objpart, k, out);
    return hipGetLastError();
}

hipError_t launch_mean_rows(const int64_t* ptr, int32_t k, int32_t* row, hipStream_t s) {
    k_mean_rows<<<grid_for(k), kThreads, 0, s>>>(ptr, k, row);
    return hipGetLastError();
}

hipError_t launch_seed_assign(const int32_t* seeds, int32_t k, int64_t n, int32_t* assign,
                              hipStream_t s) {
    k_fill_i32<<<capped(n), kThreads, 0, s>>>(assign, n, -1);
    k_scatter_seeds<<<grid_for(k), kThreads, 0, s>>>(seeds, k, n, assign);
    return hipGetLastError();
}

}  // namespace ivf
