/*
 * FP64 CPU oracle for inverted-file (IVF) spherical k-means.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call this code;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code with the GPU library.
 *
 * What it computes, in the paper's order (Aoyama, Saito, Ikeda,
 * "Inverted-File k-Means Clustering: Performance Analysis", Algorithm 3):
 *
 *  Assignment (Alg. 3, assignment step).  For each object x_i, the score
 *  vector rho of length k starts at zero.  For every nonzero (t, v) of x_i in
 *  ascending term order, the inverted-file array of term t, i.e. the list of
 *  (cluster c, mean value u) in ascending c, is walked and rho[c] += v * u
 *  (IEEE FP64, a separate multiply and add; built with -ffp-contract=off).
 *  Then rho_max starts at 0 and clusters are scanned in ascending j with a
 *  strict ">" test, so among exactly equal maxima the lowest j wins.  An
 *  object sharing no term with any mean (every rho_j == 0) keeps its previous
 *  assignment (initially -1, "unassigned").
 *
 *  Update (Alg. 3, update step).  For each cluster j with members: w = sum of
 *  member vectors in ascending object index (FP64), w <- w / |C_j|,
 *  ||w||_2 summed over ascending p, and every w_p != 0 emits
 *  (j, w_p / ||w||).  Clusters are visited in ascending j, so appending each
 *  emitted tuple to the list of term p leaves every inverted-file list in
 *  ascending cluster order.  A cluster with no member keeps its previous mean
 *  (the paper's update would divide 0 by 0 there).
 *
 *  Objective (spherical objective, Eq. sph_obj_funct): J = sum over objects,
 *  ascending i, of rho_{i, a_i} under the means the assignment used.
 *
 *  Mult-add count (Eq. ivf_mult): M = sum_i sum_h (nc)_{t(i,h)}.
 *
 * Means are handed over "mean-major": per cluster j an ascending list of
 * (term, FP64 value), CSR with int64 row pointers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Inverted file of the means: term-major lists, ascending cluster id. */
typedef struct {
    int64_t d;
    int64_t* ptr;   /* [d+1] */
    int32_t* cid;   /* [nnz] */
    double* val;    /* [nnz] */
} inv_file;

static int inv_build(inv_file* f, int64_t d, int32_t k, const int64_t* mp, const int32_t* mi,
                     const double* mv) {
    f->d = d;
    f->ptr = (int64_t*)calloc((size_t)d + 1, sizeof(int64_t));
    const int64_t nnz = mp[k];
    f->cid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    f->val = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(d > 0 ? d : 1));
    if (!f->ptr || !f->cid || !f->val || !fill) return -1;
    for (int64_t e = 0; e < nnz; ++e) f->ptr[mi[e] + 1] += 1;
    for (int64_t t = 0; t < d; ++t) f->ptr[t + 1] += f->ptr[t];
    for (int64_t t = 0; t < d; ++t) fill[t] = f->ptr[t];
    /* clusters in ascending j: each list ends up ascending in cluster id */
    for (int32_t j = 0; j < k; ++j)
        for (int64_t e = mp[j]; e < mp[j + 1]; ++e) {
            int64_t q = fill[mi[e]]++;
            f->cid[q] = j;
            f->val[q] = mv[e];
        }
    free(fill);
    return 0;
}

static void inv_free(inv_file* f) { free(f->ptr); free(f->cid); free(f->val); }

/*
 * oracle_assign: one assignment step.
 *   prev[n]        previous assignment (-1 = unassigned)
 *   out[n]         new assignment
 *   rho_a[n]       rho of the chosen cluster (0 when every rho is 0)
 *   rho_2[n]       largest rho over the other clusters (may be NULL)
 *   stats[3]       (objective J, changed count, zero-overlap count) as doubles
 *   mult[1]        M = sum_i sum_h (nc)_t
 * Returns 0, or -1 on allocation failure.
 */
int oracle_assign(int64_t n, int64_t d, const int64_t* xp, const int32_t* xi, const float* xv,
                  int32_t k, const int64_t* mp, const int32_t* mi, const double* mv,
                  const int32_t* prev, int32_t* out, double* rho_a, double* rho_2,
                  double* stats, int64_t* mult, int nthreads) {
    inv_file f;
    if (inv_build(&f, d, k, mp, mi, mv) != 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t m_total = 0, zero_total = 0, changed = 0;
    int err = 0;
    #pragma omp parallel reduction(+ : m_total, zero_total, changed)
    {
        double* rho = (double*)malloc(sizeof(double) * (size_t)k);
        if (!rho) {
            #pragma omp atomic write
            err = -1;
        } else {
            #pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < n; ++i) {
                for (int32_t j = 0; j < k; ++j) rho[j] = 0.0;
                int64_t m_i = 0;
                for (int64_t h = xp[i]; h < xp[i + 1]; ++h) {
                    const int32_t s = xi[h];
                    const double v = (double)xv[h];
                    for (int64_t q = f.ptr[s]; q < f.ptr[s + 1]; ++q) {
                        double p = v * f.val[q];
                        rho[f.cid[q]] = rho[f.cid[q]] + p;
                    }
                    m_i += f.ptr[s + 1] - f.ptr[s];
                }
                m_total += m_i;
                double best = 0.0;
                int32_t a = prev[i];
                for (int32_t j = 0; j < k; ++j)
                    if (rho[j] > best) { best = rho[j]; a = j; }
                if (best == 0.0) ++zero_total;
                double second = 0.0;
                if (rho_2) {
                    for (int32_t j = 0; j < k; ++j)
                        if (j != a && rho[j] > second) second = rho[j];
                    rho_2[i] = second;
                }
                out[i] = a;
                rho_a[i] = best;
                changed += (a != prev[i]);
            }
        }
        free(rho);
    }
    inv_free(&f);
    if (err) return err;
    double obj = 0.0;
    for (int64_t i = 0; i < n; ++i) obj += rho_a[i];
    stats[0] = obj;
    stats[1] = (double)changed;
    stats[2] = (double)zero_total;
    *mult = m_total;
    return 0;
}

/*
 * oracle_ivfd_assign: the assignment step of IVFD (Algorithm 4 of the paper),
 * which inverts the OBJECTS and queries them with each mean in turn.
 *
 * The objects' inverted file holds, for every term s, the list of
 * (object o, value u) in ascending o.  Means are visited in ascending j.  For
 * each mean the score vector rho over all N objects starts at zero (reading:
 * the printed algorithm clears rho once, before the loop over means; scores
 * of different means must not add up, so it is cleared per mean), then for
 * every term (s, v') of the mean in ascending s and every (o, u) in the list
 * of s, rho[o] = rho[o] + v' * u (FP64, separate multiply and add).  After
 * the mean, every object whose rho exceeds its running rho_max (strictly,
 * from 0) takes cluster j.  An object never raised above 0 keeps prev.
 *
 * For a fixed (object, mean) pair the products are added in ascending term
 * order, exactly as the means-inverted walk adds them, so every rho and
 * therefore the partition are bit-identical to oracle_assign's; only the loop
 * order differs.  rho_2 (largest score of any other cluster) is an extra
 * output the algorithm does not need.  Arguments as for oracle_assign;
 * single-threaded.
 */
int oracle_ivfd_assign(int64_t n, int64_t d, const int64_t* xp, const int32_t* xi,
                       const float* xv, int32_t k, const int64_t* mp, const int32_t* mi,
                       const double* mv, const int32_t* prev, int32_t* out, double* rho_a,
                       double* rho_2, double* stats, int64_t* mult) {
    const int64_t nnz = xp[n];
    int64_t* optr = (int64_t*)calloc((size_t)d + 1, sizeof(int64_t));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(d > 0 ? d : 1));
    int32_t* oobj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double* oval = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double* rho = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* second = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int err = (!optr || !fill || !oobj || !oval || !rho || !second) ? -1 : 0;
    if (!err) {
        /* inverted object file: objects in ascending i land in ascending order */
        for (int64_t e = 0; e < nnz; ++e) optr[xi[e] + 1] += 1;
        for (int64_t t = 0; t < d; ++t) optr[t + 1] += optr[t];
        for (int64_t t = 0; t < d; ++t) fill[t] = optr[t];
        for (int64_t i = 0; i < n; ++i)
            for (int64_t h = xp[i]; h < xp[i + 1]; ++h) {
                const int64_t q = fill[xi[h]]++;
                oobj[q] = (int32_t)i;
                oval[q] = (double)xv[h];
            }
        int64_t m_total = 0;
        for (int64_t i = 0; i < n; ++i) {
            rho_a[i] = 0.0;   /* rho_max */
            second[i] = 0.0;
            out[i] = prev[i];
        }
        for (int32_t j = 0; j < k; ++j) {
            for (int64_t i = 0; i < n; ++i) rho[i] = 0.0;
            for (int64_t h = mp[j]; h < mp[j + 1]; ++h) {
                const int32_t s = mi[h];
                const double v = mv[h];
                for (int64_t q = optr[s]; q < optr[s + 1]; ++q) {
                    double p = v * oval[q];
                    rho[oobj[q]] = rho[oobj[q]] + p;
                }
                m_total += optr[s + 1] - optr[s];
            }
            for (int64_t i = 0; i < n; ++i) {
                if (rho[i] > rho_a[i]) {
                    if (rho_a[i] > second[i]) second[i] = rho_a[i];
                    rho_a[i] = rho[i];
                    out[i] = j;
                } else if (rho[i] > second[i]) {
                    second[i] = rho[i];
                }
            }
        }
        int64_t zero_total = 0, changed = 0;
        double obj = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (rho_a[i] == 0.0) ++zero_total;
            changed += (out[i] != prev[i]);
            obj += rho_a[i];
            if (rho_2) rho_2[i] = second[i];
        }
        stats[0] = obj;
        stats[1] = (double)changed;
        stats[2] = (double)zero_total;
        *mult = m_total;
    }
    free(optr); free(fill); free(oobj); free(oval); free(rho); free(second);
    return err;
}

/*
 * oracle_scores: rho for listed (object, cluster) pairs, each computed by the
 * same ascending-term FP64 walk as oracle_assign (bit-identical to it).
 */
int oracle_scores(int64_t npairs, const int64_t* obj, const int32_t* clu, int64_t d,
                  const int64_t* xp, const int32_t* xi, const float* xv, int32_t k,
                  const int64_t* mp, const int32_t* mi, const double* mv, double* out) {
    inv_file f;
    if (inv_build(&f, d, k, mp, mi, mv) != 0) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npairs; ++p) {
        const int64_t i = obj[p];
        const int32_t j = clu[p];
        double acc = 0.0;
        for (int64_t h = xp[i]; h < xp[i + 1]; ++h) {
            const int32_t s = xi[h];
            const double v = (double)xv[h];
            for (int64_t q = f.ptr[s]; q < f.ptr[s + 1]; ++q)
                if (f.cid[q] == j) {
                    double pr = v * f.val[q];
                    acc = acc + pr;
                }
        }
        out[p] = acc;
    }
    inv_free(&f);
    return 0;
}

/*
 * oracle_update: one update step.
 *   assign[n]                new assignment (-1 = unassigned, ignored)
 *   pp/pi/pv                 previous means (mean-major), kept for empty clusters
 *   op[k+1], oi[cap], ov[cap] new means (mean-major), cap >= sum of output nnz
 *   sizes[k]                 |C_j|
 * Returns the output nnz (>= 0), -1 on allocation failure, -2 if cap is short.
 */
int64_t oracle_update(int64_t n, int64_t d, const int64_t* xp, const int32_t* xi, const float* xv,
                      int32_t k, const int32_t* assign, const int64_t* pp, const int32_t* pi,
                      const double* pv, int64_t* op, int32_t* oi, double* ov, int64_t cap,
                      int64_t* sizes, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t* cnt = (int64_t*)calloc((size_t)k + 1, sizeof(int64_t));
    int64_t* members = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)k + 1));
    int32_t** tidx = (int32_t**)calloc((size_t)k, sizeof(int32_t*));
    double** tval = (double**)calloc((size_t)k, sizeof(double*));
    int64_t* tlen = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    if (!cnt || !members || !fill || !tidx || !tval || !tlen) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (assign[i] >= 0) cnt[assign[i] + 1] += 1;
    for (int32_t j = 0; j < k; ++j) sizes[j] = cnt[j + 1];
    for (int32_t j = 0; j < k; ++j) cnt[j + 1] += cnt[j];
    memcpy(fill, cnt, sizeof(int64_t) * ((size_t)k + 1));
    for (int64_t i = 0; i < n; ++i)   /* members of each cluster in ascending i */
        if (assign[i] >= 0) members[fill[assign[i]]++] = i;

    int err = 0;
    #pragma omp parallel
    {
        double* w = (double*)malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
        if (!w) {
            #pragma omp atomic write
            err = -1;
        } else {
            #pragma omp for schedule(dynamic, 4)
            for (int32_t j = 0; j < k; ++j) {
                const int64_t nj = cnt[j + 1] - cnt[j];
                if (nj == 0) {            /* empty cluster: previous mean kept */
                    int64_t len = pp[j + 1] - pp[j];
                    tidx[j] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(len > 0 ? len : 1));
                    tval[j] = (double*)malloc(sizeof(double) * (size_t)(len > 0 ? len : 1));
                    memcpy(tidx[j], pi + pp[j], sizeof(int32_t) * (size_t)len);
                    memcpy(tval[j], pv + pp[j], sizeof(double) * (size_t)len);
                    tlen[j] = len;
                    continue;
                }
                for (int64_t p = 0; p < d; ++p) w[p] = 0.0;
                for (int64_t m = cnt[j]; m < cnt[j + 1]; ++m) {
                    const int64_t i = members[m];
                    for (int64_t h = xp[i]; h < xp[i + 1]; ++h)
                        w[xi[h]] = w[xi[h]] + (double)xv[h];
                }
                for (int64_t p = 0; p < d; ++p) w[p] = w[p] / (double)nj;
                double ss = 0.0;
                int64_t len = 0;
                for (int64_t p = 0; p < d; ++p) {
                    double sq = w[p] * w[p];
                    ss = ss + sq;
                    len += (w[p] != 0.0);
                }
                const double nrm = sqrt(ss);
                tidx[j] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(len > 0 ? len : 1));
                tval[j] = (double*)malloc(sizeof(double) * (size_t)(len > 0 ? len : 1));
                int64_t q = 0;
                for (int64_t p = 0; p < d; ++p)
                    if (w[p] != 0.0) {
                        tidx[j][q] = (int32_t)p;
                        tval[j][q] = w[p] / nrm;
                        ++q;
                    }
                tlen[j] = len;
            }
        }
        free(w);
    }
    int64_t total = 0;
    if (!err) {
        op[0] = 0;
        for (int32_t j = 0; j < k; ++j) {
            op[j + 1] = op[j] + tlen[j];
            total += tlen[j];
        }
        if (total > cap) err = -2;
        else
            for (int32_t j = 0; j < k; ++j) {
                memcpy(oi + op[j], tidx[j], sizeof(int32_t) * (size_t)tlen[j]);
                memcpy(ov + op[j], tval[j], sizeof(double) * (size_t)tlen[j]);
            }
    }
    for (int32_t j = 0; j < k; ++j) { free(tidx[j]); free(tval[j]); }
    free(tidx); free(tval); free(tlen); free(cnt); free(members); free(fill);
    return err ? err : total;
}

/* Term frequencies: no[t] = objects holding t; nc[t] = means holding t. */
int oracle_term_counts(int64_t n, int64_t d, const int64_t* xp, const int32_t* xi, int32_t k,
                       const int64_t* mp, const int32_t* mi, int64_t* no, int64_t* nc) {
    for (int64_t t = 0; t < d; ++t) { no[t] = 0; nc[t] = 0; }
    for (int64_t e = 0; e < xp[n]; ++e) no[xi[e]] += 1;
    for (int64_t e = 0; e < mp[k]; ++e) nc[mi[e]] += 1;
    return 0;
}
