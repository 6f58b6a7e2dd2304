// Assignment step of inverted-file spherical k-means (Algorithm 3, assignment
// part) for gfx950.
//
//   k_walk     For each (cluster range, object): stream the object's CSR
//              nonzeros, gather the range's slice of each term's posting list
//              and accumulate x_t * m_jt into the wave's own FP32 score tile
//              (ranges of up to 1,024 clusters with FP32 values: dense slabs
//              into registers, sparse slices into LDS, the two sums added once;
//              otherwise one LDS tile in ascending term order); a fused
//              wave-wide pass then extracts the range's top-1 (lowest id on
//              equal scores) and top-2 and clears the tile for the next object.
//   k_merge    Per object: merge the ranges' records, certify the FP32 argmax
//              with the rounding-error bound, else queue the object for FP64.
//   k_rescore  Per queued object: walk it again in FP32, keep the clusters the
//              bound cannot rule out, score those in FP64 exactly as the FP64
//              reference does (ascending terms, a separate multiply and add)
//              and apply the argmax rule.
//   k_objective / k_sum_final  deterministic FP64 objective and change count.
#include <algorithm>

#include "ivf_internal.h"
#include "kernels.h"

namespace ivf {
namespace {

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ inline int32_t rl32(int32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ inline int64_t rl64(int64_t x, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(x >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline float rlf(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ inline float widen16(uint32_t bits16, int vt) {
    if (vt == IVF_VAL_BF16) return __uint_as_float(bits16 << 16);
    return (float)__builtin_bit_cast(_Float16, (unsigned short)bits16);
}

// o + v * m as the walks accumulate it.  16-bit values: one fused
// multiply-add (FP16 values widen inside it, as v_fma_mix_f32), which the
// 16-bit walks, bound by VALU issue, measured 5-9 % faster with; its single
// rounding per step is within the same certification bound as a rounded
// product added with a second rounding.  FP32 values: that product and sum.
template <int VT>
__device__ inline float madd(float o, float v, float m) {
    if constexpr (VT == IVF_VAL_F32) return o + v * m;
    else return __builtin_fmaf(v, m, o);
}

// Posting entries: F32 = {cluster id, value bits}; 16-bit values = local
// cluster id (low half) | value bits (high half).
template <int VT> struct Entry;
template <> struct Entry<IVF_VAL_F32> {
    using T = uint2;
    __device__ static int32_t slot(T e, int32_t base) { return (int32_t)e.x - base; }
    __device__ static float value(T e) { return __uint_as_float(e.y); }
};
template <int VT> struct Entry16 {
    using T = uint32_t;
    __device__ static int32_t slot(T e, int32_t) { return (int32_t)(e & 0xffffu); }
    __device__ static float value(T e) { return widen16(e >> 16, VT); }
};
template <> struct Entry<IVF_VAL_BF16> : Entry16<IVF_VAL_BF16> {};
template <> struct Entry<IVF_VAL_F16> : Entry16<IVF_VAL_F16> {};

constexpr int kUnroll = 8;

// Posting-entry loads.  NT marks them non-temporal: sparse slices (tail
// terms) are rarely re-read soon, so they should not evict the head terms'
// dense slabs from L2.  That measured 2.7 % faster for the FP32 walk at 8M
// documents and 5 % slower for 16-bit values, whose smaller working set does
// reuse its sparse slices; it is used for the FP32 single-instance walk only.
template <bool NT>
__device__ inline uint2 load_entry(const uint2* p) {
    if constexpr (NT) {
        uint2 r;
        r.x = __builtin_nontemporal_load(&p->x);
        r.y = __builtin_nontemporal_load(&p->y);
        return r;
    } else {
        return *p;
    }
}
template <bool NT>
__device__ inline uint32_t load_entry(const uint32_t* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// One term's posting slice [qb, qe) accumulated into the wave's own tile:
// tile[c] = tile[c] + v * u for every entry (c, u).  LDS float atomics are
// slow on this part and not needed: the tile belongs to this wave alone, and
// one term's list names every cluster at most once, so all reads of a batch
// may be issued before its writes.  Slots are updated in ascending term order.
template <int VT, bool NT>
__device__ inline void walk_slice(const typename Entry<VT>::T* __restrict__ P, int64_t qb,
                                  int64_t qe, float v, float* tile, int32_t base, int lane) {
    using E = Entry<VT>;
    int64_t q0 = qb;
    for (; q0 + kUnroll * kWave <= qe; q0 += kUnroll * kWave) {
        typename E::T e[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) e[u] = load_entry<NT>(P + q0 + u * kWave + lane);
        float r[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) r[u] = tile[E::slot(e[u], base)];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            tile[E::slot(e[u], base)] = madd<VT>(r[u], v, E::value(e[u]));
        }
    }
    if (q0 < qe) {   // the last, partial batch: fewer than kUnroll * 64 entries
        typename E::T e[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t q = q0 + u * kWave + lane;
            ok[u] = q < qe;
            if (ok[u]) e[u] = load_entry<NT>(P + q);
        }
        float r[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (ok[u]) r[u] = tile[E::slot(e[u], base)];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (ok[u]) {
                tile[E::slot(e[u], base)] = madd<VT>(r[u], v, E::value(e[u]));
            }
    }
}

// A dense slab (the range's clusters in order, zeros for absent ones) added
// into the tile: 4 consecutive slots per lane, 128-bit LDS reads and writes.
// Adding an exact zero leaves a slot unchanged, so the tile equals the one
// the sparse slice would give.
template <int VT> struct Slab;
template <> struct Slab<IVF_VAL_F32> {
    using T = float4;
    __device__ static float4 widen(T x) { return x; }
};
template <int VT> struct Slab16 {
    using T = ushort4;
    __device__ static float4 widen(T x) {
        return make_float4(widen16(x.x, VT), widen16(x.y, VT), widen16(x.z, VT), widen16(x.w, VT));
    }
};
template <> struct Slab<IVF_VAL_BF16> : Slab16<IVF_VAL_BF16> {};
template <> struct Slab<IVF_VAL_F16> : Slab16<IVF_VAL_F16> {};

constexpr int kDenseUnroll = 4;

// A slab of at most kDenseOne * 64 groups (ranges up to 1,280 clusters) is
// walked with every global load in flight at once, then one 128-bit LDS
// read-modify-write per group: a single memory round trip per term.
constexpr int kDenseOne = 5;

template <int VT>
__device__ inline void walk_dense(const typename Slab<VT>::T* __restrict__ S, int32_t kr4, float v,
                                  float* tile, int lane) {
    using D = Slab<VT>;
    float4* t4 = reinterpret_cast<float4*>(tile);
    if (kr4 <= kDenseOne * kWave) {
        typename D::T x[kDenseOne];
#pragma unroll
        for (int u = 0; u < kDenseOne; ++u) {
            const int32_t g = u * kWave + lane;
            if (g < kr4) x[u] = S[g];
        }
#pragma unroll
        for (int u = 0; u < kDenseOne; ++u) {
            const int32_t g = u * kWave + lane;
            if (g < kr4) {
                const float4 m = D::widen(x[u]);
                float4 o = t4[g];
                o.x = madd<VT>(o.x, v, m.x);
                o.y = madd<VT>(o.y, v, m.y);
                o.z = madd<VT>(o.z, v, m.z);
                o.w = madd<VT>(o.w, v, m.w);
                t4[g] = o;
            }
        }
        return;
    }
    int32_t g0 = 0;   // groups of 4 slots; kr4 groups in the slab
    for (; g0 + kDenseUnroll * kWave <= kr4; g0 += kDenseUnroll * kWave) {
        typename D::T x[kDenseUnroll];
#pragma unroll
        for (int u = 0; u < kDenseUnroll; ++u) x[u] = S[g0 + u * kWave + lane];
        float4 r[kDenseUnroll];
#pragma unroll
        for (int u = 0; u < kDenseUnroll; ++u) r[u] = t4[g0 + u * kWave + lane];
#pragma unroll
        for (int u = 0; u < kDenseUnroll; ++u) {
            const float4 m = D::widen(x[u]);
            float4 o;
            o.x = madd<VT>(r[u].x, v, m.x);
            o.y = madd<VT>(r[u].y, v, m.y);
            o.z = madd<VT>(r[u].z, v, m.z);
            o.w = madd<VT>(r[u].w, v, m.w);
            t4[g0 + u * kWave + lane] = o;
        }
    }
    for (int32_t g = g0 + lane; g < kr4; g += kWave) {
        const float4 m = D::widen(S[g]);
        float4 o = t4[g];
        o.x = madd<VT>(o.x, v, m.x);
        o.y = madd<VT>(o.y, v, m.y);
        o.z = madd<VT>(o.z, v, m.z);
        o.w = madd<VT>(o.w, v, m.w);
        t4[g] = o;
    }
}

// Two consecutive dense terms of one object (16-bit slabs): both slabs'
// loads in flight at once, then one LDS read-modify-write per group that adds
// the first term's products and then the second's, so every slot sees the
// same additions in the same order as two single passes.  Halving the memory
// round trips made the 16-bit walks 9-10 % faster at 8M documents x
// k = 10,000; the FP32 walk, bound by L2 capacity rather than latency, was
// not faster with it.
template <int VT>
__device__ inline void walk_dense2(const typename Slab<VT>::T* __restrict__ S0,
                                   const typename Slab<VT>::T* __restrict__ S1, int32_t kr4,
                                   float v0, float v1, float* tile, int lane) {
    using D = Slab<VT>;
    float4* t4 = reinterpret_cast<float4*>(tile);
    typename D::T x0[kDenseOne], x1[kDenseOne];
#pragma unroll
    for (int u = 0; u < kDenseOne; ++u) {
        const int32_t g = u * kWave + lane;
        if (g < kr4) {
            x0[u] = S0[g];
            x1[u] = S1[g];
        }
    }
#pragma unroll
    for (int u = 0; u < kDenseOne; ++u) {
        const int32_t g = u * kWave + lane;
        if (g < kr4) {
            const float4 m0 = D::widen(x0[u]);
            const float4 m1 = D::widen(x1[u]);
            float4 o = t4[g];
            o.x = madd<VT>(o.x, v0, m0.x);
            o.y = madd<VT>(o.y, v0, m0.y);
            o.z = madd<VT>(o.z, v0, m0.z);
            o.w = madd<VT>(o.w, v0, m0.w);
            o.x = madd<VT>(o.x, v1, m1.x);
            o.y = madd<VT>(o.y, v1, m1.y);
            o.z = madd<VT>(o.z, v1, m1.z);
            o.w = madd<VT>(o.w, v1, m1.w);
            t4[g] = o;
        }
    }
}

// Wave-wide merge of (best, id, second): larger best wins, lower id on equal
// best; second collects the largest score of every other cluster.
__device__ inline void top2_combine(float& b, int32_t& id, float& s, float ob, int32_t oid,
                                    float os) {
    const bool take = ob > b || (ob == b && oid >= 0 && (id < 0 || oid < id));
    if (take) {
        s = fmaxf(os, b);
        b = ob;
        id = oid;
    } else {
        s = fmaxf(s, ob);
    }
}

// The dense slab a descriptor position p < 0 names: it starts -p - 1 values
// into the slab array.
template <int VT>
__device__ inline const typename Slab<VT>::T* slab_at(const WalkArgs& a, int64_t p) {
    return reinterpret_cast<const typename Slab<VT>::T*>(
        reinterpret_cast<const char*>(a.slab) + (-p - 1) * (VT == IVF_VAL_F32 ? 4 : 2));
}

// Object i's FP32 scores against cluster range r (clusters base .. base + kr)
// accumulated into the wave's tile, its terms in ascending order.  Returns
// the posting entries walked (the object's share of M in this range).
template <int VT, bool NT = false>
__device__ inline int32_t accumulate_object(const WalkArgs& a, int64_t i, int r, int32_t base,
                                            int32_t kr, float* tile, int lane) {
    const int64_t hb = a.x_ptr[i], he = a.x_ptr[i + 1];
    int32_t m = 0;
    for (int64_t h0 = hb; h0 < he; h0 += kWave) {
        const int cnt = (int)min((int64_t)kWave, he - h0);
        float v = 0.f;
        int32_t pos = 0, count = 0;
        if (lane < cnt) {
            const int32_t t = a.x_idx[h0 + lane];
            v = a.x_val[h0 + lane];
            const SliceDesc ds = a.desc[(int64_t)t * a.R + r];
            pos = ds.pos;
            count = ds.count;
        }
        for (int hh = 0; hh < cnt; ++hh) {
            const int64_t p = rl32(pos, hh), cn = rl32(count, hh);
            const float vv = rlf(v, hh);
            m += (int32_t)cn;
            if (p >= 0) {
                walk_slice<VT, NT>(reinterpret_cast<const typename Entry<VT>::T*>(a.post), p,
                                   p + cn, vv, tile, base, lane);
                continue;
            }
            const int32_t kr4 = (kr + 3) >> 2;
            if constexpr (VT != IVF_VAL_F32) {
                // the next term's slice is dense too: both in one pass
                if (hh + 1 < cnt && kr4 <= kDenseOne * kWave) {
                    const int64_t p1 = rl32(pos, hh + 1);
                    if (p1 < 0) {
                        m += (int32_t)rl32(count, hh + 1);
                        walk_dense2<VT>(slab_at<VT>(a, p), slab_at<VT>(a, p1), kr4, vv,
                                        rlf(v, hh + 1), tile, lane);
                        ++hh;
                        continue;
                    }
                }
            }
            walk_dense<VT>(slab_at<VT>(a, p), kr4, vv, tile, lane);
        }
    }
    return m;
}

// FP32 ranges of at most kRegClusters clusters keep the object's scores in
// registers: slots 4g .. 4g + 3 of group g = u * 64 + lane are lane's acc[u].
// A dense slab is added there with no LDS traffic; sparse slices still
// scatter into the wave's LDS tile, which is added into the registers once
// per object.  Every slot is then the sum of its dense products (ascending
// terms) plus the sum of its sparse products (ascending terms): another
// summation order of the same rounded products, so the certification bound,
// which holds for any order, is unchanged.  At 8M documents x k = 10,000
// (fixed means) the walk took 866 ms against 906 ms with the whole tile in
// LDS.  Its sparse loads are ordinary ones: the non-temporal hint that helps
// the LDS-tile walk made this one slower (906 ms).
constexpr int kRegGroups = 4;
static_assert(kRegGroups * kWave * 4 == kRegClusters, "register groups cover kRegClusters");

__device__ inline void walk_dense_reg(const float4* __restrict__ S, int32_t kr4, float v,
                                      float4 (&acc)[kRegGroups], int lane) {
    float4 x[kRegGroups];
#pragma unroll
    for (int u = 0; u < kRegGroups; ++u) {
        const int32_t g = u * kWave + lane;
        x[u] = g < kr4 ? S[g] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kRegGroups; ++u) {   // o + v * m, a product and a sum
        acc[u].x = acc[u].x + v * x[u].x;
        acc[u].y = acc[u].y + v * x[u].y;
        acc[u].z = acc[u].z + v * x[u].z;
        acc[u].w = acc[u].w + v * x[u].w;
    }
}

// Object i against range r: dense slabs into acc, sparse slices into the LDS
// tile (`sparse` tells whether any was).  Returns the entries walked.
__device__ inline int32_t accumulate_object_reg(const WalkArgs& a, int64_t i, int r, int32_t base,
                                                int32_t kr, float* tile,
                                                float4 (&acc)[kRegGroups], bool& sparse,
                                                int lane) {
    const int64_t hb = a.x_ptr[i], he = a.x_ptr[i + 1];
    const int32_t kr4 = (kr + 3) >> 2;
    int32_t m = 0;
    for (int64_t h0 = hb; h0 < he; h0 += kWave) {
        const int cnt = (int)min((int64_t)kWave, he - h0);
        float v = 0.f;
        int32_t pos = 0, count = 0;
        if (lane < cnt) {
            const int32_t t = a.x_idx[h0 + lane];
            v = a.x_val[h0 + lane];
            const SliceDesc ds = a.desc[(int64_t)t * a.R + r];
            pos = ds.pos;
            count = ds.count;
        }
        for (int hh = 0; hh < cnt; ++hh) {
            const int64_t p = rl32(pos, hh), cn = rl32(count, hh);
            const float vv = rlf(v, hh);
            m += (int32_t)cn;
            if (p >= 0) {
                sparse = true;
                walk_slice<IVF_VAL_F32, false>(reinterpret_cast<const uint2*>(a.post), p, p + cn,
                                               vv, tile, base, lane);
            } else {
                walk_dense_reg(slab_at<IVF_VAL_F32>(a, p), kr4, vv, acc, lane);
            }
        }
    }
    return m;
}

// One work item of an FP32 range of at most kRegClusters clusters: per object
// the register walk, the sparse sums added (the LDS tile cleared), top-1 and
// top-2 over the registers and the range record.
__device__ inline void walk_item_reg(const WalkArgs& a, int64_t w, float* tile, int lane) {
    const int r = (int)(w / a.items_per_range);
    const int64_t c = w - (int64_t)r * a.items_per_range;
    const int32_t base = r * a.k_r;
    const int32_t kr = min(a.k_r, a.k - base);
    const int32_t kr4 = (kr + 3) >> 2;
    const int64_t i0 = c * a.chunk;
    const int64_t i1 = min(a.n, i0 + a.chunk);
    float4* t4 = reinterpret_cast<float4*>(tile);
    for (int64_t i = i0; i < i1; ++i) {
        float4 acc[kRegGroups];
#pragma unroll
        for (int u = 0; u < kRegGroups; ++u) acc[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        bool sparse = false;
        const int32_t m = accumulate_object_reg(a, i, r, base, kr, tile, acc, sparse, lane);
        if (sparse) {
#pragma unroll
            for (int u = 0; u < kRegGroups; ++u) {
                const int32_t g = u * kWave + lane;
                if (g < kr4) {
                    const float4 q = t4[g];
                    t4[g] = make_float4(0.f, 0.f, 0.f, 0.f);
                    acc[u].x = acc[u].x + q.x;
                    acc[u].y = acc[u].y + q.y;
                    acc[u].z = acc[u].z + q.z;
                    acc[u].w = acc[u].w + q.w;
                }
            }
        }
        // top-2 in ascending slot order per lane, then across lanes
        float b = 0.f, s2 = 0.f;
        int32_t id = -1;
#pragma unroll
        for (int u = 0; u < kRegGroups; ++u) {
            const int32_t s0 = (u * kWave + lane) * 4;
            const float x[4] = {acc[u].x, acc[u].y, acc[u].z, acc[u].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (s0 + e < kr) {
                    if (x[e] > b) {
                        s2 = fmaxf(s2, b);
                        b = x[e];
                        id = s0 + e;
                    } else {
                        s2 = fmaxf(s2, x[e]);
                    }
                }
            }
        }
#pragma unroll
        for (int o = kWave / 2; o >= 1; o >>= 1) {
            const float ob = __shfl_xor(b, o, kWave);
            const int32_t oid = __shfl_xor(id, o, kWave);
            const float os = __shfl_xor(s2, o, kWave);
            top2_combine(b, id, s2, ob, oid, os);
        }
        RangeRec rec;
        rec.best = b;
        rec.id = id >= 0 ? base + id : -1;
        rec.second = s2;
        rec.m = m;
        a.rec[(int64_t)r * a.n + i] = rec;
    }
}

// One work item: `chunk` consecutive objects against cluster range r, each
// walked into the wave's tile, its range record written and the tile cleared.
template <int VT, bool NT = false>
__device__ inline void walk_item(const WalkArgs& a, int64_t w, float* tile, int lane) {
    const int r = (int)(w / a.items_per_range);
    const int64_t c = w - (int64_t)r * a.items_per_range;
    const int32_t base = r * a.k_r;
    const int32_t kr = min(a.k_r, a.k - base);
    const int64_t i0 = c * a.chunk;
    const int64_t i1 = min(a.n, i0 + a.chunk);
    for (int64_t i = i0; i < i1; ++i) {
        const int32_t m = accumulate_object<VT, NT>(a, i, r, base, kr, tile, lane);
        // fused top-2 over the tile, clearing it for the next object
        float b = 0.f, s2 = 0.f;
        int32_t id = -1;
        for (int s0 = lane * 4; s0 < kr; s0 += 4 * kWave) {
            const float4 q = *reinterpret_cast<const float4*>(tile + s0);
            *reinterpret_cast<float4*>(tile + s0) = make_float4(0.f, 0.f, 0.f, 0.f);
            const float x[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (x[u] > b) {
                    s2 = fmaxf(s2, b);
                    b = x[u];
                    id = s0 + u;
                } else {
                    s2 = fmaxf(s2, x[u]);
                }
            }
        }
#pragma unroll
        for (int o = kWave / 2; o >= 1; o >>= 1) {
            const float ob = __shfl_xor(b, o, kWave);
            const int32_t oid = __shfl_xor(id, o, kWave);
            const float os = __shfl_xor(s2, o, kWave);
            top2_combine(b, id, s2, ob, oid, os);
        }
        // every lane holds the same record: identical stores, no divergence
        RangeRec rec;
        rec.best = b;
        rec.id = id >= 0 ? base + id : -1;
        rec.second = s2;
        rec.m = m;
        a.rec[(int64_t)r * a.n + i] = rec;
    }
}

__device__ inline void zero_tile(float* tile, int stride, int lane) {
    for (int s = lane * 4; s < stride; s += 4 * kWave)
        *reinterpret_cast<float4*>(tile + s) = make_float4(0.f, 0.f, 0.f, 0.f);
}

// The whole wave claims its next work item: one atomic from lane 0, whose
// result every lane takes with readfirstlane after the lanes reconverge, so
// the caller's loop test is scalar and all 64 lanes leave the loop together.
__device__ inline int64_t claim_item(unsigned long long* ctr, int lane) {
    unsigned long long v = 0ull;
    if (lane == 0) v = atomicAdd(ctr, 1ull);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Waves per SIMD the walk is compiled for (the register budget): 8 for 16-bit
// values (about a dozen registers spill; 7, without spills, measured no faster);
// 6 for the FP32 LDS-tile walk (8 measured 18 % slower: it is bound by L2
// capacity, not by latency hiding); 7 for the FP32 register walk, whose
// registers then hold 3 workgroups of 8 waves as at 6 (28 waves in 4-wave
// workgroups and 32 at 8 per SIMD were no faster).
constexpr int walk_waves_per_eu(int vt, bool reg) {
    return vt != IVF_VAL_F32 ? 8 : (reg ? 7 : 6);
}

// REG: the FP32 register walk (every range of at most kRegClusters clusters).
template <int VT, bool REG>
__global__ __launch_bounds__(kWave * kMaxWaves)
__attribute__((amdgpu_waves_per_eu(walk_waves_per_eu(VT, REG), 8))) void k_walk(WalkArgs a) {
    extern __shared__ float4 lds4[];
    const int lane = lane_id();
    // wave index made provably uniform, so every loop below has uniform bounds
    // and cross-lane reads always see all 64 lanes active
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    float* tile = reinterpret_cast<float*>(lds4) + (int64_t)wv * a.tile_stride;
    zero_tile(tile, a.tile_stride, lane);
    const int64_t total = a.items_per_range * a.R;
    // items in ascending order, claimed from the counter: all waves sweep the
    // ranges in the same order and stay within one window of consecutive
    // items, so a range's slices stay hot in the caches (against a static
    // round robin at 8M documents x k = 10,000: FP32 2 % faster, 16-bit 14 %)
    for (;;) {
        const int64_t w = claim_item(&a.cnt->work, lane);
        if (w >= total) break;
        if constexpr (REG) walk_item_reg(a, w, tile, lane);
        else walk_item<VT, VT == IVF_VAL_F32>(a, w, tile, lane);
    }
}

// Many instances in one persistent launch: item w belongs to the instance b
// with item_off[b] <= w < item_off[b + 1]; every wave's tile holds the widest
// range of all instances.  Items are claimed from a counter in ascending
// order: items of different instances cost very different amounts, and a
// static round robin let the waves drift apart across ranges and instances
// (a working set many times one range's); claiming keeps all waves within
// one window of consecutive items.  Every claim advances the counter, so a
// wave leaves after at most total + 1 claims.  The FP32 kernel is compiled
// for 6 waves per SIMD (1.2 % faster than 7 on the 96-instance mix), the
// 16-bit ones for 7.  FP32 instances take the register walk exactly when a
// single handle of the same plan would (ranges of at most kRegClusters), so
// a batch computes each instance's scores as its own handle does; ALLREG
// marks a batch whose instances all do.
template <int VT, bool ALLREG>
__global__ __launch_bounds__(kWave * kMaxWaves)
__attribute__((amdgpu_waves_per_eu(VT == IVF_VAL_F32 ? 6 : 7, 8))) void k_walk_batch(const WalkArgs* __restrict__ args,
                                                                  const int64_t* __restrict__ item_off,
                                                                  int32_t count, int32_t tile_stride,
                                                                  unsigned long long* work) {
    extern __shared__ float4 lds4[];
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    float* tile = reinterpret_cast<float*>(lds4) + (int64_t)wv * tile_stride;
    zero_tile(tile, tile_stride, lane);
    const int64_t total = item_off[count];
    for (;;) {
        const int64_t w = claim_item(work, lane);
        if (w >= total) break;
        int32_t lo = 0, hi = count;   // last b with item_off[b] <= w
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (item_off[mid] <= w) lo = mid; else hi = mid;
        }
        const WalkArgs a = args[lo];
        if constexpr (VT == IVF_VAL_F32 && ALLREG) {
            walk_item_reg(a, w - item_off[lo], tile, lane);
        } else if constexpr (VT == IVF_VAL_F32) {
            if (a.k_r <= kRegClusters) walk_item_reg(a, w - item_off[lo], tile, lane);
            else walk_item<VT>(a, w - item_off[lo], tile, lane);
        } else {
            walk_item<VT>(a, w - item_off[lo], tile, lane);
        }
    }
}

constexpr int kMergeBlock = 256;

// Objects in a grid-stride loop; the counters reduced per thread, per wave and
// per block, then added with one atomic per block and counter.  One atomic
// per wave on the same four addresses (125,000 waves at 8M objects) queued
// for 3 ms on one L2 channel.
__global__ __launch_bounds__(kMergeBlock) void k_merge(MergeArgs a) {
    int64_t m = 0;                          // entries walked (M)
    uint32_t n_cert = 0, n_zero = 0;        // certified and zero-overlap objects
    double rel = 0.0;                       // largest relative bound of a kept FP32 winner
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float b = 0.f, s2 = 0.f;
        int32_t id = -1;
        int64_t mi = 0;
        for (int r = 0; r < a.R; ++r) {
            const RangeRec rec = a.rec[(int64_t)r * a.n + i];
            mi += rec.m;
            // ranges arrive in ascending cluster order: an equal best keeps the earlier
            if (rec.best > b) {
                s2 = fmaxf(fmaxf(s2, b), rec.second);
                b = rec.best;
                id = rec.id;
            } else {
                s2 = fmaxf(s2, rec.best);
            }
        }
        m += mi;
        const int32_t prev = a.prev[i];
        a.best[i] = b;
        a.best_id[i] = id;
        a.second[i] = s2;
        uint8_t flag;
        if (mi == 0) {                     // no term shared with any mean
            a.assign[i] = prev;
            a.rho[i] = 0.0;
            flag = 4;
            ++n_zero;
        } else {
            double c, ab, g;
            if (a.fixed_scale > 0.0)
                cert_consts_fixed(a.x_ptr[i + 1] - a.x_ptr[i], a.fixed_scale, a.vmax, &c, &ab,
                                  &g);
            else
                cert_consts(a.valtype, a.x_ptr[i + 1] - a.x_ptr[i], a.vmax, &c, &ab, &g);
            // a non-finite score certifies nothing (the library rejects inputs
            // whose FP32 scores could overflow; this keeps the rule total)
            const bool ok = !a.force_rescore && b > 0.f && isfinite(b) && isfinite(s2) &&
                            cert_lb((double)b, c, ab, g) > cert_ub((double)s2, c, ab, g);
            if (ok || !a.certify) {
                a.assign[i] = id >= 0 ? id : prev;
                a.rho[i] = (double)b;
                flag = ok ? 1 : 0;
                n_cert += ok ? 1u : 0u;
                rel = fmax(rel, c + (ab > 0.0 && b > 0.f ? ab / (double)b : 0.0));
            } else {
                const unsigned long long slot = atomicAdd(&a.cnt->n_rescore, 1ull);
                a.rescore_list[slot] = (int32_t)i;
                flag = 2;
            }
        }
        a.flags[i] = flag;
    }
    // integer sums and a maximum: the same in any order (non-negative
    // doubles order like their bit patterns)
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        m += __shfl_xor(m, o, kWave);
        n_cert += __shfl_xor(n_cert, o, kWave);
        n_zero += __shfl_xor(n_zero, o, kWave);
        rel = fmax(rel, __shfl_xor(rel, o, kWave));
    }
    constexpr int W = kMergeBlock / kWave;
    __shared__ int64_t s_m[W];
    __shared__ uint32_t s_cert[W], s_zero[W];
    __shared__ double s_rel[W];
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s_m[w] = m;
        s_cert[w] = n_cert;
        s_zero[w] = n_zero;
        s_rel[w] = rel;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < W; ++q) {
            m += s_m[q];
            n_cert += s_cert[q];
            n_zero += s_zero[q];
            rel = fmax(rel, s_rel[q]);
        }
        if (m) atomicAdd(&a.cnt->mult, (unsigned long long)m);
        if (n_cert) atomicAdd(&a.cnt->certified, (unsigned long long)n_cert);
        if (n_zero) atomicAdd(&a.cnt->zero_overlap, (unsigned long long)n_zero);
        if (rel > 0.0)
            atomicMax(&a.cnt->max_bound_bits, (unsigned long long)__double_as_longlong(rel));
    }
}

// FP64 score of cluster j for the object with nonzeros [hb, he), exactly as
// the FP64 reference computes it: the products v * u in ascending term order,
// each a separate FP64 multiply, added one after another (a term absent from
// mean j adds an exact zero).  u comes from mean j's FP64 row.  The sum runs
// in a wave-uniform loop, so every lane holds the same value.
__device__ inline double exact_score(const RescoreArgs& a, int64_t hb, int64_t he, int32_t j,
                                     int lane) {
    const int64_t rb = a.mm_ptr[j], re = a.mm_ptr[j + 1];
    double sum = 0.0;
    for (int64_t h0 = hb; h0 < he; h0 += kWave) {
        const int cnt = (int)min((int64_t)kWave, he - h0);
        double p = 0.0;
        if (lane < cnt) {
            const int32_t t = a.w.x_idx[h0 + lane];
            int64_t lo = rb, hi = re;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (a.mm_idx[mid] < t) lo = mid + 1; else hi = mid;
            }
            if (lo < re && a.mm_idx[lo] == t) p = (double)a.w.x_val[h0 + lane] * a.mm_val[lo];
        }
        for (int hh = 0; hh < cnt; ++hh)
            sum = sum + __longlong_as_double(rl64(__double_as_longlong(p), hh));
    }
    return sum;
}

// Objects the FP32 bound could not certify, one per wave.  A cluster j is a
// candidate unless the bounds prove it below the FP32 winner (each score
// within its own walk's bound of the FP64 one): every non-candidate's FP64
// score is then strictly smaller than the winner's, so the FP64 argmax
// (lowest j on equal scores) is among the candidates.  Candidates get their
// exact FP64 score and, in ascending j with a strict test from 0, the
// reference's rule picks the cluster.
// The walk's record of each range bounds its scores: its best is the range
// winner's, its second the largest of every other cluster's.  A range whose
// best cannot be a candidate is skipped; one whose second cannot be holds one
// candidate, its winner; any other range is walked again in FP32 into the
// LDS tile and its candidates read from the tile.  Without records (another
// walk's), every range is walked.  Where the main walk kept a range's scores
// in registers, the walk again adds the same products in another order, so
// its scores may differ from the walk's in the last bits; each is within its
// own bound of the FP64 score, which is all the rule above uses.
template <int VT>
__global__ __launch_bounds__(kWave * kMaxWaves) void k_rescore(RescoreArgs a) {
    extern __shared__ float4 lds4[];
    const WalkArgs& w = a.w;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
    float* tile = reinterpret_cast<float*>(lds4) + (int64_t)wv * w.tile_stride;
    zero_tile(tile, w.tile_stride, lane);
    const int64_t nq = (int64_t)a.cnt->n_rescore;
    for (int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv; q < nq; q += nwaves) {
        const int64_t i = a.rescore_list[q];
        const int64_t hb = w.x_ptr[i], he = w.x_ptr[i + 1];
        const int32_t prev = a.prev[i];
        const int32_t fw = a.best_id[i];
        double c, ab, g;
        cert_consts(a.valtype, he - hb, a.vmax, &c, &ab, &g);
        // the winner's score may come from another walk (IVFD's fixed-point
        // sums): its lower bound then uses that walk's constants
        double thr;
        if (a.fixed_scale > 0.0) {
            double c1, ab1, g1;
            cert_consts_fixed(he - hb, a.fixed_scale, a.vmax, &c1, &ab1, &g1);
            thr = cert_lb((double)a.best[i], c1, ab1, g1);
        } else {
            thr = cert_lb((double)a.best[i], c, ab, g);
        }
        double best = 0.0;
        int32_t bj = prev;
        double rho_fw = -1.0;   // FP64 score of the FP32 winner (always a candidate)
        for (int r = 0; r < w.R; ++r) {
            const int32_t base = r * w.k_r;
            const int32_t kr = min(w.k_r, w.k - base);
            if (a.rec) {
                const RangeRec rr = a.rec[(int64_t)r * w.n + i];
                if (cert_ub((double)rr.best, c, ab, g) < thr) continue;
                if (rr.id >= 0 && cert_ub((double)rr.second, c, ab, g) < thr) {
                    const double e = exact_score(a, hb, he, rr.id, lane);
                    if (e > best) {
                        best = e;
                        bj = rr.id;
                    }
                    if (rr.id == fw) rho_fw = e;
                    continue;
                }
            }
            accumulate_object<VT>(w, i, r, base, kr, tile, lane);
            for (int s0 = 0; s0 < kr; s0 += 4 * kWave) {
                const int s = s0 + 4 * lane;
                float4 q4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (s < kr) {
                    q4 = *reinterpret_cast<const float4*>(tile + s);
                    *reinterpret_cast<float4*>(tile + s) = make_float4(0.f, 0.f, 0.f, 0.f);
                }
                const float x[4] = {q4.x, q4.y, q4.z, q4.w};
                uint64_t mk[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    mk[u] = __ballot(s + u < kr && cert_ub((double)x[u], c, ab, g) >= thr);
                uint64_t any = mk[0] | mk[1] | mk[2] | mk[3];
                while (any) {   // uniform: ascending lanes, then the lane's 4 slots
                    const int l = __builtin_ctzll(any);
                    any &= any - 1;
                    for (int u = 0; u < 4; ++u) {
                        if (!((mk[u] >> l) & 1ull)) continue;
                        const int32_t j = base + s0 + 4 * l + u;
                        const double e = exact_score(a, hb, he, j, lane);
                        if (e > best) {
                            best = e;
                            bj = j;
                        }
                        if (j == fw) rho_fw = e;
                    }
                }
            }
        }
        // best, bj and rho_fw are wave-uniform: identical stores from every
        // lane, and an idempotent max
        a.assign[i] = best > 0.0 ? bj : prev;
        a.rho[i] = best;
        if (rho_fw > 0.0) {
            const double e = fabs((double)a.best[i] - rho_fw) / rho_fw;
            atomicMax(&a.cnt->max_err_bits, (unsigned long long)__double_as_longlong(e));
        }
    }
}

// Deterministic FP64 sum of rho over fixed chunks + change count.
__global__ __launch_bounds__(256) void k_objective(const double* __restrict__ rho,
                                                   const int32_t* __restrict__ assign,
                                                   const int32_t* __restrict__ prev, int64_t n,
                                                   int64_t per_block, double* __restrict__ part,
                                                   Counters* cnt) {
    __shared__ double sh[256];
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = min(n, b0 + per_block);
    double acc = 0.0;
    unsigned long long ch = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        acc += rho[i];
        ch += (assign[i] != prev[i]);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
    if (ch) atomicAdd(&cnt->changed, ch);
}

__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ part, int64_t m,
                                                   double* __restrict__ out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_zero_u64(unsigned long long* p) {
    if (threadIdx.x == 0) *p = 0ull;
}

__global__ void k_clear_counters(Counters* c) {
    unsigned long long* p = reinterpret_cast<unsigned long long*>(c);
    const int n = (int)(sizeof(Counters) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

}  // namespace

hipError_t launch_clear_counters(Counters* c, hipStream_t s) {
    k_clear_counters<<<1, 64, 0, s>>>(c);
    return hipGetLastError();
}

hipError_t launch_walk(const WalkArgs& a, int valtype, int waves, int lds_bytes, int grid,
                       hipStream_t s) {
    const dim3 blk(kWave * waves);
    if (valtype == IVF_VAL_F32 && a.k_r <= kRegClusters)
        k_walk<IVF_VAL_F32, true><<<grid, blk, lds_bytes, s>>>(a);
    else if (valtype == IVF_VAL_F32)
        k_walk<IVF_VAL_F32, false><<<grid, blk, lds_bytes, s>>>(a);
    else if (valtype == IVF_VAL_BF16)
        k_walk<IVF_VAL_BF16, false><<<grid, blk, lds_bytes, s>>>(a);
    else
        k_walk<IVF_VAL_F16, false><<<grid, blk, lds_bytes, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_walk_batch(const WalkArgs* args, const int64_t* item_off, int32_t count,
                             int32_t tile_stride, int valtype, int waves, int grid,
                             unsigned long long* work, hipStream_t s) {
    const dim3 blk(kWave * waves);
    const size_t lds = (size_t)waves * tile_stride * 4;
    k_zero_u64<<<1, 64, 0, s>>>(work);
    if (valtype == IVF_VAL_F32 && tile_stride <= kRegClusters)
        k_walk_batch<IVF_VAL_F32, true><<<grid, blk, lds, s>>>(args, item_off, count, tile_stride,
                                                               work);
    else if (valtype == IVF_VAL_F32)
        k_walk_batch<IVF_VAL_F32, false><<<grid, blk, lds, s>>>(args, item_off, count, tile_stride,
                                                                work);
    else if (valtype == IVF_VAL_BF16)
        k_walk_batch<IVF_VAL_BF16, false><<<grid, blk, lds, s>>>(args, item_off, count,
                                                                 tile_stride, work);
    else
        k_walk_batch<IVF_VAL_F16, false><<<grid, blk, lds, s>>>(args, item_off, count,
                                                                tile_stride, work);
    return hipGetLastError();
}

const void* walk_kernel_ptr(int valtype, int32_t k_r) {
    if (valtype == IVF_VAL_F32 && k_r <= kRegClusters)
        return reinterpret_cast<const void*>(&k_walk<IVF_VAL_F32, true>);
    if (valtype == IVF_VAL_F32) return reinterpret_cast<const void*>(&k_walk<IVF_VAL_F32, false>);
    if (valtype == IVF_VAL_BF16)
        return reinterpret_cast<const void*>(&k_walk<IVF_VAL_BF16, false>);
    return reinterpret_cast<const void*>(&k_walk<IVF_VAL_F16, false>);
}

const void* walk_batch_kernel_ptr(int valtype, int32_t tile_stride) {
    if (valtype == IVF_VAL_F32 && tile_stride <= kRegClusters)
        return reinterpret_cast<const void*>(&k_walk_batch<IVF_VAL_F32, true>);
    if (valtype == IVF_VAL_F32)
        return reinterpret_cast<const void*>(&k_walk_batch<IVF_VAL_F32, false>);
    if (valtype == IVF_VAL_BF16)
        return reinterpret_cast<const void*>(&k_walk_batch<IVF_VAL_BF16, false>);
    return reinterpret_cast<const void*>(&k_walk_batch<IVF_VAL_F16, false>);
}

hipError_t walk_set_lds_limit(int lds_bytes) {
    // the attribute is per kernel and shared by every handle: allow the whole
    // LDS, each launch asks for what its tiles need
    lds_bytes = kLdsBytes;
    const void* ks[] = {walk_kernel_ptr(IVF_VAL_F32, kRegClusters),
                        walk_kernel_ptr(IVF_VAL_F32, kRegClusters + 1),
                        walk_kernel_ptr(IVF_VAL_BF16, 0),
                        walk_kernel_ptr(IVF_VAL_F16, 0),
                        walk_batch_kernel_ptr(IVF_VAL_F32, kRegClusters),
                        walk_batch_kernel_ptr(IVF_VAL_F32, kRegClusters + 1),
                        walk_batch_kernel_ptr(IVF_VAL_BF16, 0),
                        walk_batch_kernel_ptr(IVF_VAL_F16, 0)};
    for (const void* k : ks) {
        hipError_t e =
            hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    for (int vt = IVF_VAL_F32; vt <= IVF_VAL_F16; ++vt) {
        hipError_t e = hipFuncSetAttribute(rescore_kernel_ptr(vt),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

const void* rescore_kernel_ptr(int valtype) {
    if (valtype == IVF_VAL_F32) return reinterpret_cast<const void*>(&k_rescore<IVF_VAL_F32>);
    if (valtype == IVF_VAL_BF16) return reinterpret_cast<const void*>(&k_rescore<IVF_VAL_BF16>);
    return reinterpret_cast<const void*>(&k_rescore<IVF_VAL_F16>);
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
    // eight blocks per CU at most; every object is one thread's in the loop
    const int64_t blocks = std::min<int64_t>((a.n + kMergeBlock - 1) / kMergeBlock, 2048);
    if (blocks > 0) k_merge<<<(unsigned)blocks, kMergeBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_rescore(const RescoreArgs& a, int waves, int grid, hipStream_t s) {
    const dim3 blk(kWave * waves);
    const size_t lds = (size_t)waves * a.w.tile_stride * 4;
    if (a.valtype == IVF_VAL_F32)
        k_rescore<IVF_VAL_F32><<<grid, blk, lds, s>>>(a);
    else if (a.valtype == IVF_VAL_BF16)
        k_rescore<IVF_VAL_BF16><<<grid, blk, lds, s>>>(a);
    else
        k_rescore<IVF_VAL_F16><<<grid, blk, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_objective(const double* rho, const int32_t* assign, const int32_t* prev,
                            int64_t n, double* part, int nblocks, double* out, Counters* cnt,
                            hipStream_t s) {
    if (n <= 0) {
        k_sum_final<<<1, 256, 0, s>>>(part, 0, out);
        return hipGetLastError();
    }
    const int64_t per = (n + nblocks - 1) / nblocks;
    k_objective<<<nblocks, 256, 0, s>>>(rho, assign, prev, n, per, part, cnt);
    k_sum_final<<<1, 256, 0, s>>>(part, nblocks, out);
    return hipGetLastError();
}

}  // namespace ivf
