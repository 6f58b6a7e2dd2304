// IVFD: the assignment step with the OBJECTS inverted (the paper's
// Algorithm 4, Section "IVFD and IVF").  Every mean is a query over the
// objects' inverted file; its scores for all objects fill an N-vector, and
// each object then compares that score with its running maximum (strict
// ">", means in ascending j, from 0).
//
// On this part the N-vector is tiled: a workgroup owns a range of n_r
// objects (one score slot per object in LDS) and a block of consecutive
// means, and walks each mean over the slice of the objects' inverted file
// that falls into its range.  The file is therefore stored range-major: for
// range r and term s the entries {object within the range, FP32 value} of the
// objects of r holding s, in ascending object order, bounded by
// optr[r * d + s] .. optr[r * d + s + 1].
//
// A mean's terms are taken 1024 at a time (one per thread): each thread loads
// its term's slice bounds, a workgroup scan lays the nonempty slices end to
// end and the 16 waves split the concatenation evenly, so short slices (most
// of them: a range holds few objects of a term) still fill all 64 lanes.
// Different terms reach the same object, so the adds into the shared tile
// are LDS atomics, and in fixed point: an FP32 float atomic add to LDS runs
// at a thirtieth of the rate of a 32-bit integer one on this part.  Each
// product is scaled by 2^F and rounded to an integer; F is chosen from the
// largest object and mean norms so that no score's sum can exceed 2^32.  The
// integer sums are exact and independent of the order of the adds; the
// certification bound accounts for the rounding (relative, from the FP32
// products; absolute, half a unit of 2^-F per product).  The running (best,
// cluster, second) of the workgroup's objects live in registers as integers.
#include "kernels.h"

namespace ivf {
namespace {

constexpr int kThreads = 256;
constexpr int kIvfdThreads = 1024;
constexpr int kIvfdWaves = kIvfdThreads / kWave;
constexpr int kIvfdUnroll = 8;

inline unsigned grid_for(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20));
}

// Sort keys of the build: (range, term) of every object entry.
__global__ void k_ivfd_keys(const int32_t* __restrict__ rowid, const int32_t* __restrict__ x_idx,
                            int64_t nnz, int32_t n_r, int64_t d, uint32_t* __restrict__ keys) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        keys[e] = (uint32_t)((int64_t)(rowid[e] / n_r) * d + x_idx[e]);
}

// Slice bounds from the sorted keys: optr[key] = first entry whose key is
// >= key, for every key in [0, nkeys].  Entry e fills the keys after its
// predecessor's key up to its own.
__global__ void k_ivfd_bounds(const uint32_t* __restrict__ keys, int64_t nnz, int64_t nkeys,
                              uint32_t* __restrict__ optr) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e <= nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = e == 0 ? 0 : (int64_t)keys[e - 1] + 1;
        const int64_t hi = e == nnz ? nkeys : (int64_t)keys[e];
        for (int64_t q = lo; q <= hi; ++q) optr[q] = (uint32_t)e;
    }
}

// Entries in (range, term, object) order: {object - range start, value bits}.
__global__ void k_ivfd_post(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ pos,
                            const int32_t* __restrict__ rowid, const float* __restrict__ x_val,
                            int64_t nnz, int32_t n_r, int64_t d, uint2* __restrict__ post) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = pos[q];
        const int64_t r = (int64_t)keys[q] / d;
        post[q] = make_uint2((uint32_t)(rowid[e] - r * n_r), __float_as_uint(x_val[e]));
    }
}

// Entries every object meets over all means: the sum over its terms of the
// number of means holding the term (the object's share of M, saturated at
// 2^31 - 1; zero exactly when it shares no term with any mean), in the first
// of its B records (0 in the others).
__global__ void k_ivfd_overlap(const int64_t* __restrict__ x_ptr,
                               const int32_t* __restrict__ x_idx, int64_t n, int32_t B,
                               const int64_t* __restrict__ ivf_ptr, RangeRec* __restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t m = 0;
    for (int64_t h = x_ptr[i]; h < x_ptr[i + 1]; ++h) {
        const int32_t t = x_idx[h];
        m += ivf_ptr[t + 1] - ivf_ptr[t];
    }
    rec[i].m = (int32_t)std::min<int64_t>(m, 0x7fffffff);
    for (int32_t b = 1; b < B; ++b) rec[(int64_t)b * n + i].m = 0;
}

// Largest row norm, FP64 sums of squares in row order.
__global__ void k_max_row_norm(const int64_t* __restrict__ ptr, const float* __restrict__ v32,
                               const double* __restrict__ v64, int64_t rows,
                               unsigned long long* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    double s = 0.0;
    for (int64_t h = ptr[i]; h < ptr[i + 1]; ++h) {
        const double v = v64 ? v64[h] : (double)v32[h];
        s = s + v * v;
    }
    if (s > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(sqrt(s)));
}

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(x, o, kWave);
        if (lane >= o) x += t;
    }
    return x;
}

// First l in [lo, nt) with t_incl[l] > q, given t_incl[nt - 1] > q and
// t_incl[lo - 1] <= q: a galloping search from lo (cheap when q has moved
// past few slices, logarithmic when it has moved past many).
__device__ inline int next_slice(const uint32_t* t_incl, int lo, int nt, uint32_t q) {
    int step = 1, hi = lo;
    while (t_incl[hi] <= q) {
        lo = hi + 1;
        hi = min(lo + step - 1, nt - 1);
        step <<= 1;
    }
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t_incl[mid] > q) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// One workgroup per (range of NR = 4096 * G objects, block of means); 4 G
// objects per thread.
template <int G>
__global__ __launch_bounds__(kIvfdThreads) void k_ivfd_walk(IvfdArgs a) {
    constexpr int NR = 4096 * G;
    constexpr int S = 4 * G;   // objects per thread
    extern __shared__ uint4 lds_u4[];
    uint32_t* tile = reinterpret_cast<uint32_t*>(lds_u4);
    uint32_t* t_incl = tile + NR;                 // inclusive ends of the nonempty slices
    uint32_t* t_off = t_incl + kIvfdThreads;      // entry = t_off + position
    float* t_v = reinterpret_cast<float*>(t_off + kIvfdThreads);   // the term's mean value
    uint32_t* w_sum = reinterpret_cast<uint32_t*>(t_v + kIvfdThreads);   // [2 * kIvfdWaves + 2]
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int r = blockIdx.x / a.B;
    const int b = blockIdx.x - r * a.B;
    const int32_t kb = (a.k + a.B - 1) / a.B;
    const int32_t j0 = b * kb, j1 = min(a.k, j0 + kb);
    const uint32_t* __restrict__ optr = a.optr + (int64_t)r * a.d;

    uint32_t best[S], sec[S];
    int32_t bid[S];
#pragma unroll
    for (int u = 0; u < S; ++u) {
        best[u] = 0u;
        sec[u] = 0u;
        bid[u] = -1;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) lds_u4[tid + kIvfdThreads * g] = make_uint4(0u, 0u, 0u, 0u);
    unsigned long long walked = 0;
    __syncthreads();

    for (int32_t j = j0; j < j1; ++j) {
        const int64_t jb = a.mm_ptr[j], je = a.mm_ptr[j + 1];
        for (int64_t sb = jb; sb < je; sb += kIvfdThreads) {
            // this thread's term: its slice in the range and the mean's value
            const int64_t h = sb + tid;
            uint32_t c = 0, p0 = 0;
            float v = 0.f;
            if (h < je) {
                const int32_t s = a.mm_idx[h];
                v = (float)a.mm_val[h];
                p0 = optr[s];
                c = optr[s + 1] - p0;
            }
            // workgroup scans of the slice lengths and of the nonempty flags
            const uint32_t f = c > 0 ? 1u : 0u;
            uint32_t incl = wave_incl_scan(c, lane);
            uint32_t fincl = wave_incl_scan(f, lane);
            if (lane == kWave - 1) {
                w_sum[wv] = incl;
                w_sum[kIvfdWaves + wv] = fincl;
            }
            __syncthreads();
            if (wv == 0) {
                const uint32_t t = lane < kIvfdWaves ? w_sum[lane] : 0u;
                const uint32_t tf = lane < kIvfdWaves ? w_sum[kIvfdWaves + lane] : 0u;
                const uint32_t ti = wave_incl_scan(t, lane);
                const uint32_t tfi = wave_incl_scan(tf, lane);
                if (lane < kIvfdWaves) {
                    w_sum[lane] = ti - t;
                    w_sum[kIvfdWaves + lane] = tfi - tf;
                }
                if (lane == kIvfdWaves - 1) {
                    w_sum[2 * kIvfdWaves] = ti;
                    w_sum[2 * kIvfdWaves + 1] = tfi;
                }
            }
            __syncthreads();
            incl += w_sum[wv];
            if (f) {   // nonempty slices only, in term order
                const uint32_t slot = fincl + w_sum[kIvfdWaves + wv] - 1;
                t_incl[slot] = incl;
                t_off[slot] = p0 - (incl - c);   // modulo 2^32: p0 + (position - slice start)
                t_v[slot] = v;
            }
            const uint32_t T = w_sum[2 * kIvfdWaves];
            const int nt = (int)w_sum[2 * kIvfdWaves + 1];
            __syncthreads();
            if (tid == 0) walked += T;
            // this wave's share [qa, qb) of the concatenated slices
            const uint32_t qa = (uint32_t)(((uint64_t)T * wv) / kIvfdWaves);
            const uint32_t qb = (uint32_t)(((uint64_t)T * (wv + 1)) / kIvfdWaves);
            if (qa < qb) {
                // t_incl[nt - 1] == T > every position below qb, so each
                // search ends inside [0, nt)
                int l = next_slice(t_incl, 0, nt, min(qa + lane, qb - 1));
                for (uint32_t q0 = qa; q0 < qb; q0 += kWave * kIvfdUnroll) {
                    uint2 e[kIvfdUnroll];
                    float vv[kIvfdUnroll];
#pragma unroll
                    for (int u = 0; u < kIvfdUnroll; ++u) {
                        const uint32_t q = q0 + u * kWave + lane;
                        vv[u] = 0.f;
                        e[u] = make_uint2(0u, 0u);
                        if (q < qb) {
                            if (t_incl[l] <= q) l = next_slice(t_incl, l + 1, nt, q);
                            vv[u] = t_v[l];
                            e[u] = a.opost[t_off[l] + q];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kIvfdUnroll; ++u) {
                        const uint32_t q = q0 + u * kWave + lane;
                        if (q < qb) {
                            const float p = vv[u] * __uint_as_float(e[u].y);
                            atomicAdd(tile + e[u].x, __float2uint_rn(p * a.scale));
                        }
                    }
                }
            }
            __syncthreads();   // tables reused by the next batch; the tile complete after the last
        }
        // the running maxima of this thread's objects; the tile cleared
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int gi = tid + kIvfdThreads * g;
            const uint4 t = lds_u4[gi];
            lds_u4[gi] = make_uint4(0u, 0u, 0u, 0u);
            const uint32_t x[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int sl = 4 * g + u;
                if (x[u] > best[sl]) {
                    sec[sl] = max(sec[sl], best[sl]);
                    best[sl] = x[u];
                    bid[sl] = j;
                } else {
                    sec[sl] = max(sec[sl], x[u]);
                }
            }
        }
        __syncthreads();   // cleared before the next mean adds into it
    }
    const int64_t obj0 = (int64_t)r * NR;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t o = obj0 + 4 * (int64_t)(tid + kIvfdThreads * g) + u;
            if (o < a.n) {
                RangeRec* p = a.rec + (int64_t)b * a.n + o;
                // an integer sum converted once (FP32 rounding) and scaled by 2^-F
                p->best = (float)best[4 * g + u] * a.inv_scale;
                p->id = bid[4 * g + u];
                p->second = (float)sec[4 * g + u] * a.inv_scale;
            }
        }
    if (tid == 0 && walked) atomicAdd(a.walked, walked);
}

const void* ivfd_kernel(int g) {
    if (g == 1) return reinterpret_cast<const void*>(&k_ivfd_walk<1>);
    if (g == 2) return reinterpret_cast<const void*>(&k_ivfd_walk<2>);
    return reinterpret_cast<const void*>(&k_ivfd_walk<4>);
}

}  // namespace

int ivfd_lds_bytes(int32_t n_r) {
    return n_r * 4 + 3 * kIvfdThreads * 4 + (2 * kIvfdWaves + 2) * 4;
}

hipError_t launch_ivfd_build(const int32_t* rowid, const int32_t* x_idx, const float* x_val,
                             int64_t nnz, int32_t n_r, int64_t d, int64_t nkeys, uint32_t* keys,
                             uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                             const uint32_t* iota, void* tmp, uint32_t* optr, uint2* post,
                             hipStream_t s) {
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) <= nkeys - 1) ++bits;
    if (nnz > 0) {
        k_ivfd_keys<<<grid_for(nnz), kThreads, 0, s>>>(rowid, x_idx, nnz, n_r, d, keys);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = radix_sort_pairs(keys, vals, keys_alt, vals_alt, nnz, bits, tmp, s, iota);
        if (e != hipSuccess) return e;
    }
    k_ivfd_bounds<<<grid_for(nnz + 1), kThreads, 0, s>>>(keys, nnz, nkeys, optr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nnz == 0) return e;
    k_ivfd_post<<<grid_for(nnz), kThreads, 0, s>>>(keys, vals, rowid, x_val, nnz, n_r, d, post);
    return hipGetLastError();
}

hipError_t launch_ivfd_walk(const IvfdArgs& a, hipStream_t s) {
    const int g = a.n_r / 4096;
    if (a.n_r != 4096 * g || (g != 1 && g != 2 && g != 4)) return hipErrorInvalidValue;
    const int lds = ivfd_lds_bytes(a.n_r);
    hipError_t e = hipFuncSetAttribute(ivfd_kernel(g), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       lds);
    if (e != hipSuccess) return e;
    if (a.B < 1 || (int64_t)a.R * a.B >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(a.R * a.B);
    if (g == 1) k_ivfd_walk<1><<<grid, kIvfdThreads, lds, s>>>(a);
    else if (g == 2) k_ivfd_walk<2><<<grid, kIvfdThreads, lds, s>>>(a);
    else k_ivfd_walk<4><<<grid, kIvfdThreads, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_ivfd_overlap(const int64_t* x_ptr, const int32_t* x_idx, int64_t n, int32_t B,
                               const int64_t* ivf_ptr, RangeRec* rec, hipStream_t s) {
    k_ivfd_overlap<<<grid_for(n), kThreads, 0, s>>>(x_ptr, x_idx, n, B, ivf_ptr, rec);
    return hipGetLastError();
}

hipError_t launch_max_row_norm(const int64_t* ptr, const float* val32, const double* val64,
                               int64_t rows, unsigned long long* out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_max_row_norm<<<grid_for(rows), kThreads, 0, s>>>(ptr, val32, val64, rows, out);
    return hipGetLastError();
}

}  // namespace ivf
