// Device-wide exclusive scan and stable LSD radix sort of (uint32 key, uint32
// value) pairs for gfx950.  Both are building blocks of the update step
// (grouping object entries by cluster) and of the inverted-file transpose
// (grouping mean entries by term), which need stable, deterministic orders.
#include <algorithm>

#include "ivf_internal.h"

namespace ivf {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;      // 4096 items per block

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

template <typename T>
__device__ inline T wave_inclusive_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan over the block; *total receives the block sum.
template <typename T>
__device__ inline T block_exclusive_scan(T x, T* sh, T* total) {
    const int lane = lane_id(), w = threadIdx.x / kWave;
    T inc = wave_inclusive_scan(x);
    if (lane == kWave - 1) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int i = 0; i < kBlock / kWave; ++i) {
            T t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[kBlock / kWave] = acc;
    }
    __syncthreads();
    T res = inc - x + sh[w];
    *total = sh[kBlock / kWave];
    __syncthreads();
    return res;
}

// Tile totals: consecutive threads read consecutive elements (the sum of
// integers does not depend on the order).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const T* __restrict__ in, int64_t n,
                                                      T* __restrict__ sums) {
    __shared__ T sh[kBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int64_t q = base + i * kBlock + threadIdx.x;
        acc += q < n ? in[q] : (T)0;
    }
    T total;
    block_exclusive_scan(acc, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Position of tile element e in the LDS staging array: one pad slot per 16
// elements, so that the 16-element chunks the threads scan are read and
// written without bank conflicts.
__device__ inline int staged(int e) { return e + (e >> 4); }

// Exclusive scan of one tile (plus the tile's offset): the tile is loaded
// coalesced into LDS, each thread scans its chunk of kItems consecutive
// elements, and the results go back through LDS to coalesced stores.  in and
// out may be the same array (each tile is read whole before it is written).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const T* __restrict__ in, T* __restrict__ out,
                                                      int64_t n, const T* __restrict__ offs) {
    __shared__ T sh[kBlock / kWave + 1];
    __shared__ T tile[kTile + kTile / 16];
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int e = i * kBlock + threadIdx.x;
        const int64_t q = base + e;
        tile[staged(e)] = q < n ? in[q] : (T)0;
    }
    __syncthreads();
    T v[kItems];
    T acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = tile[staged(threadIdx.x * kItems + i)];
        acc += v[i];
    }
    T total;
    T run = block_exclusive_scan(acc, sh, &total);   // synchronises the block
    if (offs) run += offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        tile[staged(threadIdx.x * kItems + i)] = run;
        run += v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int e = i * kBlock + threadIdx.x;
        const int64_t q = base + e;
        if (q < n) out[q] = tile[staged(e)];
    }
}

inline int64_t ntiles(int64_t n) { return (n + kTile - 1) / kTile; }

template <typename T>
size_t scan_levels_bytes(int64_t n) {
    size_t b = 0;
    while (n > kTile) {
        n = ntiles(n);
        b += ((size_t)n * sizeof(T) + 255) & ~(size_t)255;
    }
    return b;
}

template <typename T>
hipError_t scan_impl(const T* in, T* out, int64_t n, void* tmp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = ntiles(n);
    if (nb == 1) {
        k_tile_scan<T><<<1, kBlock, 0, s>>>(in, out, n, nullptr);
        return hipGetLastError();
    }
    T* sums = reinterpret_cast<T*>(tmp);
    void* rest = reinterpret_cast<char*>(tmp) + (((size_t)nb * sizeof(T) + 255) & ~(size_t)255);
    k_tile_sums<T><<<(unsigned)nb, kBlock, 0, s>>>(in, n, sums);
    hipError_t e = scan_impl<T>(sums, sums, nb, rest, s);
    if (e != hipSuccess) return e;
    k_tile_scan<T><<<(unsigned)nb, kBlock, 0, s>>>(in, out, n, sums);
    return hipGetLastError();
}

// ------------------------------------------------------------- radix sort
// A tile of kSortTile items per block; digits of DB bits (8, or 9 where that
// saves a pass), each thread owning kDig / kSortBlock consecutive digits.
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kMaxDigitBits = 9;

inline int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

template <int DB>
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                           int64_t n, const int64_t* n_dev,
                                                           int shift, uint32_t* __restrict__ hist,
                                                           int64_t nt) {
    constexpr int D = 1 << DB, P = D / kSortBlock;
    static_assert(P >= 1 && P * kSortBlock == D, "whole digits per thread");
    __shared__ uint32_t h[D];
    n = bounded_count(n, n_dev);
#pragma unroll
    for (int u = 0; u < P; ++u) h[threadIdx.x * P + u] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + (int64_t)r * kSortBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (D - 1)], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const int d = threadIdx.x * P + u;
        hist[(int64_t)d * nt + blockIdx.x] = h[d];
    }
}

// Stable scatter of one tile of kSortTile items.  Wave w ranks the items w *
// kSortTile/4 .. (w + 1) * kSortTile/4 - 1 of the tile, 64 consecutive ones
// per round, against counters of its own (peers of a digit found by DB
// ballots), so no barrier is needed while ranking; the waves' counts then
// give every digit's run in the tile.  The keys are placed in LDS in digit
// order and written out run by run (consecutive threads write consecutive
// addresses of a run, where writing each item straight to its bucket touched
// one cache line per item); the values then go through the same LDS buffer
// to the places their keys went.  One buffer for both keeps the block at 37
// KB of LDS with 8-bit digits (42 KB with 9-bit ones), four (three) blocks
// per CU, enough waves in flight to cover the latency of the loads and
// stores.  Ranks follow (wave, round, lane), the input order, so the pass is
// stable.  The tile's count of digit d is the difference of consecutive
// entries of the scanned histogram (laid out digit-major, tile-minor), the
// last entry's against n.
template <typename V, int DB>
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(
    const uint32_t* __restrict__ keys, const V* __restrict__ vals, int64_t n,
    const int64_t* n_dev, int shift, const uint32_t* __restrict__ offs, int64_t nt,
    uint32_t* __restrict__ okeys, V* __restrict__ ovals) {
    constexpr int D = 1 << DB, P = D / kSortBlock;
    constexpr int W = kSortBlock / kWave;
    constexpr int R = kSortItems;          // rounds per wave (64 items each)
    constexpr uint32_t kNone = 0xffffffffu;
    static_assert(P >= 1 && P * kSortBlock == D, "whole digits per thread");
    static_assert(sizeof(V) % sizeof(uint32_t) == 0, "values are whole words");
    n = bounded_count(n, n_dev);
    __shared__ V stage[kSortTile];         // the tile's keys, then its values
    __shared__ uint32_t wcnt[W][D];        // per wave: its items of each digit so far
    __shared__ uint32_t to_glob[D];        // global start minus tile start of each digit's run
    uint32_t* s_keys = reinterpret_cast<uint32_t*>(stage);
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
#pragma unroll
    for (int q = 0; q < W; ++q)
#pragma unroll
        for (int u = 0; u < P; ++u) wcnt[q][tid * P + u] = 0u;
    uint32_t start[P];                     // tile start of the runs of this thread's digits
    {
        uint32_t g[P], cnt[P], sum = 0;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int64_t idx = (int64_t)(tid * P + u) * nt + blockIdx.x;
            g[u] = offs[idx];
            const uint32_t next = idx + 1 < (int64_t)D * nt ? offs[idx + 1] : (uint32_t)n;
            cnt[u] = next - g[u];
            sum += cnt[u];
        }
        uint32_t total;
        // the staging buffer is free until the placement: scratch of the scan
        uint32_t st = block_exclusive_scan<uint32_t>(sum, s_keys, &total);
#pragma unroll
        for (int u = 0; u < P; ++u) {
            start[u] = st;
            // >= 0: earlier digits hold at least this tile's items
            to_glob[tid * P + u] = g[u] - st;
            st += cnt[u];
        }
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)w * (R * kWave);
    uint32_t key[R], rk[R];
    V val[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = base + r * kWave + lane;
        const bool valid = i < n;
        key[r] = valid ? keys[i] : 0u;
        if (valid) val[r] = vals[i];
        const uint32_t d = (key[r] >> shift) & (D - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt);
        const uint32_t c = wcnt[w][d];   // read by every peer before the first of them adds
        rk[r] = valid ? c + before : kNone;
        if (valid && before == 0) wcnt[w][d] = c + (uint32_t)__popcll(peers);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < P; ++u) {   // per digit: the waves' offsets inside its run
        const int d = tid * P + u;
        uint32_t acc = start[u];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const uint32_t t = wcnt[q][d];
            wcnt[q][d] = acc;
            acc += t;
        }
    }
    __syncthreads();
    // keys in digit order; rk becomes each item's place in the tile
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (rk[r] != kNone) {
            const uint32_t d = (key[r] >> shift) & (D - 1);
            const uint32_t pos = wcnt[w][d] + rk[r];
            rk[r] = pos < (uint32_t)kSortTile ? pos : kNone;
            if (pos < (uint32_t)kSortTile) s_keys[pos] = key[r];
        }
    }
    __syncthreads();
    // the tile in digit order: runs of consecutive addresses; each thread
    // keeps the global places of the slots it wrote for the values' pass
    const int64_t tbase = (int64_t)blockIdx.x * kSortTile;
    const int items = (int)std::min<int64_t>(kSortTile, std::max<int64_t>(0, n - tbase));
    uint32_t gpos[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int p = i * kSortBlock + tid;
        gpos[i] = kNone;
        if (p < items) {
            const uint32_t k2 = s_keys[p];
            const int64_t pos = (int64_t)to_glob[(k2 >> shift) & (D - 1)] + p;
            if (pos < n) {
                okeys[pos] = k2;
                gpos[i] = (uint32_t)pos;
            }
        }
    }
    __syncthreads();   // every key read before the values take the buffer
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (rk[r] != kNone) stage[rk[r]] = val[r];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int p = i * kSortBlock + tid;
        if (p < items && gpos[i] != kNone) ovals[gpos[i]] = stage[p];
    }
}

// The result of an odd number of passes copied back (a kernel, so the sort
// records no memory-copy node of host-chosen size when captured in a graph).
template <typename V>
__global__ void k_copy2(const uint32_t* __restrict__ a, const V* __restrict__ b,
                        uint32_t* __restrict__ oa, V* __restrict__ ob, int64_t n,
                        const int64_t* n_dev) {
    n = bounded_count(n, n_dev);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        oa[i] = a[i];
        ob[i] = b[i];
    }
}

// Positions and histogram offsets are 32-bit: n stays below 2^32 - 1 (the
// value that marks an empty slot in the scatter).
constexpr int64_t kSortMax = (int64_t)0xffffffffu - 1;

template <typename V, int DB>
hipError_t radix_pass(const uint32_t* ki, const V* vin, uint32_t* ko, V* vo, int64_t n,
                      const int64_t* n_dev, int shift, uint32_t* hist, void* stmp, int64_t nt,
                      hipStream_t s) {
    k_radix_hist<DB><<<(unsigned)nt, kSortBlock, 0, s>>>(ki, n, n_dev, shift, hist, nt);
    hipError_t e = scan_impl<uint32_t>(hist, hist, nt * ((int64_t)1 << DB), stmp, s);
    if (e != hipSuccess) return e;
    k_radix_scatter<V, DB><<<(unsigned)nt, kSortBlock, 0, s>>>(ki, vin, n, n_dev, shift, hist, nt,
                                                               ko, vo);
    return hipGetLastError();
}

template <typename V>
hipError_t radix_sort_impl(uint32_t* keys, V* vals, uint32_t* keys_alt, V* vals_alt, int64_t n,
                           int bits, void* tmp, hipStream_t s, const V* vals_in_first,
                           const int64_t* n_dev) {
    if (n <= 0) return hipSuccess;
    if (n > kSortMax) return hipErrorInvalidValue;
    if (bits < 1) bits = 1;
    const int64_t nt = sort_tiles(n);
    uint32_t* hist = reinterpret_cast<uint32_t*>(tmp);
    void* stmp = reinterpret_cast<char*>(tmp) +
                 (((size_t)nt * (1 << kMaxDigitBits) * sizeof(uint32_t) + 255) & ~(size_t)255);
    // 8-bit digits, except that keys of 17 or 18 bits take two passes of 9
    // bits (the inverted file's term keys: no third pass and no copy back)
    const int db = (bits > 16 && bits <= 2 * kMaxDigitBits) ? kMaxDigitBits : 8;
    const int passes = (bits + db - 1) / db;
    uint32_t *ki = keys, *ko = keys_alt;
    V *vi = vals, *vo = vals_alt;
    for (int p = 0; p < passes; ++p) {
        const int shift = db * p;
        const V* vin = (p == 0 && vals_in_first) ? vals_in_first : vi;
        const hipError_t e =
            db == 8 ? radix_pass<V, 8>(ki, vin, ko, vo, n, n_dev, shift, hist, stmp, nt, s)
                    : radix_pass<V, kMaxDigitBits>(ki, vin, ko, vo, n, n_dev, shift, hist, stmp,
                                                   nt, s);
        if (e != hipSuccess) return e;
        uint32_t* t = ki; ki = ko; ko = t;
        V* tv = vi; vi = vo; vo = tv;
    }
    if (ki != keys) {   // odd number of passes: move the result home
        k_copy2<V><<<(unsigned)std::min<int64_t>(nt * kSortItems, 65536), kSortBlock, 0, s>>>(
            ki, vi, keys, vals, n, n_dev);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) { return scan_levels_bytes<int64_t>(n) + 256; }

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp,
                              hipStream_t s) {
    return scan_impl<uint32_t>(in, out, n, tmp, s);
}

hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp,
                              hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, tmp, s);
}

size_t radix_tmp_bytes(int64_t n) {
    const int64_t nt = sort_tiles(n > 0 ? n : 1);
    const int64_t entries = nt * ((int64_t)1 << kMaxDigitBits);
    const size_t hist = ((size_t)entries * sizeof(uint32_t) + 255) & ~(size_t)255;
    return hist + scan_levels_bytes<uint32_t>(entries) + 256;
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                            uint32_t* vals_alt, int64_t n, int bits, void* tmp, hipStream_t s,
                            const uint32_t* vals_in_first, const int64_t* n_dev) {
    return radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s,
                                     vals_in_first, n_dev);
}

hipError_t radix_sort_pairs_u64(uint32_t* keys, uint2* vals, uint32_t* keys_alt, uint2* vals_alt,
                                int64_t n, int bits, void* tmp, hipStream_t s,
                                const uint2* vals_in_first, const int64_t* n_dev) {
    return radix_sort_impl<uint2>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s, vals_in_first,
                                  n_dev);
}

}  // namespace ivf
