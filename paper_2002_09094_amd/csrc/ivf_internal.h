// Internal declarations of the gfx950 IVF spherical k-means library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/ivf.h"

namespace ivf {

constexpr int kWave = 64;
constexpr int kLdsBytes = 160 * 1024;      // LDS per CU (and per workgroup) on gfx950
constexpr int kMaxWaves = 16;
// FP32 cluster ranges of at most this many clusters take the register walk
// (each lane holds 16 of the range's scores in registers).
constexpr int32_t kRegClusters = 1024;

// Launch plan of the assignment walk (chosen by make_plan).
struct Plan {
    int32_t k = 0;
    int32_t k_r = 0;          // clusters per FP32 score tile (one range)
    int32_t R = 0;            // number of cluster ranges
    int32_t waves = 0;        // waves per workgroup, each owning one tile
    int32_t chunk = 0;        // objects per work-queue item
    int32_t tile_stride = 0;  // floats per tile (k_r rounded up to a multiple of 4)
    int32_t k_r64 = 0;        // clusters per range of the FP64 re-score (its FP32 candidate walk)
    int32_t R64 = 0;
    int32_t lds_bytes = 0;    // per workgroup of the walk
};

// One (term, cluster range) slice of the inverted file.  pos >= 0: sparse,
// entries [pos, pos + count) of the posting array; pos < 0: dense slab of the
// range's width at element offset -pos - 1 of the slab array.  count is the
// number of clusters of the range holding the term either way.  8 bytes: the
// posting array holds fewer than 2^31 entries and the slab array fewer than
// 2^31 - 1 elements (the rebuild keeps a slice sparse rather than exceed it).
struct SliceDesc {
    int32_t pos;
    int32_t count;
};
constexpr int64_t kMaxSlabElems = ((int64_t)1 << 31) - 256;

// Per (object, range) result of the walk.
struct RangeRec {
    float best;      // largest tile score in the range (0 if none)
    int32_t id;      // its cluster id (global), -1 if best == 0
    float second;    // largest score of any other cluster of the range
    int32_t m;       // posting entries walked for this object in this range
};

// Device-side counters, cleared by a kernel before each step.
struct Counters {
    unsigned long long work;        // walk work queue
    unsigned long long work64;      // re-score work queue
    unsigned long long n_rescore;   // flagged objects
    unsigned long long mult;        // posting entries walked
    unsigned long long certified;
    unsigned long long zero_overlap;
    unsigned long long changed;
    unsigned long long empty;
    unsigned long long max_err_bits;   // max relative error (double bits, >= 0)
    unsigned long long max_bound_bits; // max objective bound (double bits, >= 0)
    unsigned long long error_flags;    // validation
    unsigned long long walked;         // entries the IVFD walk met
    unsigned long long norm_bits;      // largest row norm (double bits, >= 0)
    unsigned long long inexact;        // terms whose fixed-point member sums are rounded
    unsigned long long vmax_bits;      // validation: largest value (double bits, >= 0)
    unsigned long long nmax;           // validation: longest row
};

// Error flags raised by the validation kernels.
enum : unsigned {
    kBadPtr = 1u,
    kBadIndex = 2u,
    kBadOrder = 4u,
    kNonFinite = 8u,
    kNonPositive = 16u,
    kOverflow = 32u,   // new means exceeded a fixed capacity
};

// Entry count of a capacity-bounded launch: the device-side count when it
// fits the capacity n, else 0 (a producer that overflowed wrote nothing valid).
__device__ inline int64_t bounded_count(int64_t n, const int64_t* n_dev) {
    if (!n_dev) return n;
    const int64_t v = *n_dev;
    return (v >= 0 && v <= n) ? v : 0;
}

// Absolute rounding terms of the certificate.  kEtaF32: the largest error of
// one FP32 (or BF16) rounding of a result below the normal range, whether it
// is kept as a subnormal (at most 2^-150) or flushed to zero (below 2^-126);
// 2^-126 covers both.  kEtaF16: half the smallest FP16 subnormal, the error of
// rounding a mean value below FP16's normal range (the library is built with
// FP16 denormals kept).
constexpr double kEtaF32 = 0x1p-126;
constexpr double kEtaF16 = 0x1p-25;

// Certification constants: see ivf_cert_bound in ivf.h.  vmax bounds every
// object value.  Per product of the walk: the stored mean value differs from
// the FP64 one by at most u_s relatively plus eta_m absolutely (below the
// stored type's normal range), scaled by the object value (<= vmax); the
// product's and the sum's roundings add u relatively and eta absolutely each.
__host__ __device__ inline void cert_consts(int valtype, int64_t nt, double vmax, double* c,
                                            double* a, double* g64) {
    const double u32 = 0x1p-24, u64 = 0x1p-53;
    double us, eta_m;
    if (valtype == IVF_VAL_F32) {
        us = u32;
        eta_m = kEtaF32;
    } else if (valtype == IVF_VAL_BF16) {
        us = 0x1p-8 + u32 + 0x1p-32;   // FP64 -> FP32 -> BF16
        eta_m = kEtaF32;
    } else {
        us = 0x1p-11 + u32 + 0x1p-35;  // FP64 -> FP32 -> FP16
        eta_m = kEtaF16 + kEtaF32;
    }
    const double n = (double)(nt > 0 ? nt : 1);
    const double g32 = n * u32 / (1.0 - n * u32);
    double cc = (1.0 + us) * (1.0 + g32) - 1.0;
    *c = cc * 1.01 + 1e-15;
    *a = n * (vmax * eta_m + 2.0 * kEtaF32) * (1.0 + g32) * 1.01;
    *g64 = (n * u64 / (1.0 - n * u64)) * 1.01 + 1e-17;
}

// Bound constants of a score summed in fixed point: the product of the
// FP32-rounded mean value and the FP32 object value, rounded in FP32, scaled
// by `scale` (a power of two) and rounded to the nearest integer; the nt
// integers summed exactly; the sum converted to FP32 and divided by scale.
// Relative: the two FP32 roundings before the sum and the one after; absolute:
// half a unit of 1 / scale per product, plus the FP32 roundings of the mean
// value (times the object value, <= vmax) and of the product below the normal
// range.  g64 as for cert_consts.
__host__ __device__ inline void cert_consts_fixed(int64_t nt, double scale, double vmax,
                                                  double* c, double* a, double* g64) {
    const double u32 = 0x1p-24, u64 = 0x1p-53;
    const double n = (double)(nt > 0 ? nt : 1);
    const double cc = (1.0 + u32) * (1.0 + u32) * (1.0 + u32) - 1.0;
    *c = cc * 1.01 + 1e-15;
    *a = n * (0.5 / scale + (vmax + 1.0) * kEtaF32) * (1.0 + u32) * 1.01;
    *g64 = (n * u64 / (1.0 - n * u64)) * 1.01 + 1e-17;
}

__host__ __device__ inline double cert_lb(double s, double c, double a, double g) {
    return (s - a) * (1.0 - g) / (1.0 + c);
}
__host__ __device__ inline double cert_ub(double s, double c, double a, double g) {
    return (s + a) * (1.0 + g) / (1.0 - c);
}

// ----------------------------------------------------------------- primitives
// Exclusive scan of n values (uint32 or int64) in place or out of place.
// tmp must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp,
                              hipStream_t s);
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp,
                              hipStream_t s);

// Stable LSD radix sort of (key, value) uint32 pairs on bits [0, bits).
// Buffers: keys/vals are in-out (result lands back in keys/vals);
// keys_alt/vals_alt are scratch of n entries; tmp holds radix_tmp_bytes(n).
// If vals_in_first != nullptr, the first pass reads values from it instead
// of vals (saves a copy of an immutable payload).  If n_dev != nullptr, the
// number of pairs is min(n, *n_dev), read on the device (n is the capacity).
size_t radix_tmp_bytes(int64_t n);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                            uint32_t* vals_alt, int64_t n, int bits, void* tmp, hipStream_t s,
                            const uint32_t* vals_in_first = nullptr,
                            const int64_t* n_dev = nullptr);
// The same with 8-byte values (the whole payload moves with its key).
hipError_t radix_sort_pairs_u64(uint32_t* keys, uint2* vals, uint32_t* keys_alt, uint2* vals_alt,
                                int64_t n, int bits, void* tmp, hipStream_t s,
                                const uint2* vals_in_first = nullptr,
                                const int64_t* n_dev = nullptr);

// Plan of the walk for k clusters.
ivf_status make_plan(int32_t k, const ivf_options* o, Plan* p, std::string* err);
// Default dense-slab threshold of a plan (a slice holding at least this share
// of its range's clusters is stored as a dense slab).
float dense_default(int32_t valtype, int32_t k_r);

}  // namespace ivf
