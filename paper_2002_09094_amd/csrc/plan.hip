// Launch plan of the assignment walk: cluster-range width, waves per
// workgroup, objects per work item, and the dense-slab threshold of the
// inverted file the walk reads.  The plan decides what the walk's kernels do
// and therefore what their hardware counters read.
#include "ivf_internal.h"

namespace ivf {

// Default share of a range's clusters from which a (term, range) slice is a
// dense slab.  The LDS-tile walks: 0.35, measured fastest at 8M documents x
// k = 10,000 (FP32 LDS-tile walk: 936 ms against 962 ms at 0.5 and 995 ms at
// 0.2; BF16 670 against 677 ms; FP16 flat).  The FP32 register walk: 0.45
// (same workload, fixed means after 4 and after 8 iterations: 847 and 849 ms
// against 865 and 895 ms at 0.35, 881 and 902 ms at 0.5 and 0.48; on the
// 2M-document k = 50,000 workload 1,509 against 1,492 ms at 0.35).
float dense_default(int32_t valtype, int32_t k_r) {
    return (valtype == IVF_VAL_F32 && k_r <= kRegClusters) ? 0.45f : 0.35f;
}

ivf_status make_plan(int32_t k, const ivf_options* o, Plan* p, std::string* err) {
    if (k < 1) {
        if (err) *err = "k must be >= 1";
        return IVF_ERR_ARG;
    }
    // Widest tile: 1024 clusters for FP32 values, 1280 for 16-bit ones (whose
    // dense slabs are half the bytes), with 8 tiles per workgroup, measured
    // best at 8M documents x k = 10,000 (FP32: 922 ms at 1000-cluster ranges
    // against 935 ms at 1250 and 964 ms at 834; BF16: 655 ms at 1250 against
    // 683 ms at 1000).  The hot set of a range, the dense slabs of its head
    // terms, then about fills one XCD's 4 MB L2.
    const int32_t vt = o ? o->valtype : IVF_VAL_F32;
    int32_t kr_max = (o && o->cluster_range > 0) ? o->cluster_range
                                                 : (vt == IVF_VAL_F32 ? 1024 : 1280);
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
    // 8 objects per work item: with items claimed from a counter, one object
    // per item made the counter a bottleneck (FP32 walk at 8M documents 7 %
    // slower); 2 to 32 measured the same
    q.chunk = (o && o->objects_per_item > 0) ? o->objects_per_item : 8;
    q.k_r64 = q.k_r;   // the FP64 re-score walks the same ranges
    q.R64 = q.R;
    *p = q;
    return IVF_OK;
}

}  // namespace ivf
