/*
 * gini_oracle.c -- plain single-threaded FP64 reference for Gini MDS.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file or the library built from it: only the test-suite, the
 * package's smoke check and the benchmark's CPU-baseline leg use it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Every function follows the paper (arXiv 2605.25124, "Optimizing
 * Multidimensional Scaling in Gini Metric Spaces") in its own order and
 * notation; the section or equation is named above each one.  No blocking,
 * fusion, vectorisation or reordering is applied.  The only memoisation is
 * a per-call table of F^{nu-1} for the 2d-1 possible (doubled) ranks, which
 * returns the very same pow() results the loop would compute.
 *
 * Readings taken where the paper is silent or garbled (each one is also
 * listed in the design notes):
 *   R1  ties get midranks, R(v_c) = #{v < v_c} + (#{v == v_c} + 1) / 2
 *       (tied values share the midpoint of their ranks, as Section III-A
 *       intends; the printed tie formula is garbled).
 *       Ranks are returned doubled, t = 2R, so that they are integers.
 *   R2  inside the generalised distance of Section III-B the survival function
 *       of a coordinate of the compared difference vector is the empirical
 *       one over its d coordinates, Fbar(z_c) = 1 - R(z_c)/d, and
 *       Fbar(0) = 1 - R(0)/d with R(0) = (d+1)/2 (as for the Gini norm).
 *   R3  the factor d multiplying the sum is the length of the compared vectors.
 *   R4  the latent distance is selectable: the Gini pseudo-distance itself
 *       (Section IV-B fits a Gini metric space) or the Euclidean norm
 *       (Algorithm 1 evaluates the fit with Euclidean latent distances).
 *   R5  the minimised loss is the raw stress sum_{i<j} (delta_ij - Delta_ij)^2
 *       (the SMACOF loss of Section IV-B with unit weights).
 *   R6  ranks are held fixed when differentiating (the distance is piecewise
 *       linear in the data), which gives the gradient almost everywhere.
 *   R7  the fixed step is eta = eta_s / (2 n c) with c = |d delta / d u|^2 for
 *       a tie-free u (c = 1 for the Euclidean latent: the Guttman step).
 *   R8  MATCH32 mode decides every rank on the same FP32 bits as a single
 *       precision device: z_c = fl32(fl32(x_ic) - fl32(x_jc)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXACT 0
#define ORC_MATCH32 1
#define ORC_LATENT_GINI 0
#define ORC_LATENT_EUCLID 1

/* ------------------------------------------------------------------ ranks */

/* Definition 1 (rank within one vector) with the midrank reading R1 for ties,
 * written straight from the definition by counting: O(d^2). */
void orc_rank2_count(const double* v, int d, int32_t* t) {
    for (int c = 0; c < d; ++c) {
        int less = 0, eq = 0;
        for (int k = 0; k < d; ++k) {
            if (v[k] < v[c]) ++less;
            else if (v[k] == v[c]) ++eq;
        }
        t[c] = 2 * less + eq + 1;
    }
}

typedef struct { double v; int32_t i; } orc_vi;

static int orc_cmp_vi(const void* a, const void* b) {
    const orc_vi* x = (const orc_vi*)a;
    const orc_vi* y = (const orc_vi*)b;
    if (x->v < y->v) return -1;
    if (y->v < x->v) return 1;
    return (x->i > y->i) - (x->i < y->i);
}

/* Same ranks by sorting: a run of equal values occupying sorted positions
 * a..b (0-based) holds 1-based ranks a+1..b+1, whose mean doubled is a+b+2. */
void orc_rank2_sort(const double* v, int d, int32_t* t) {
    orc_vi* s = (orc_vi*)malloc(sizeof(orc_vi) * (size_t)(d > 0 ? d : 1));
    for (int c = 0; c < d; ++c) { s[c].v = v[c]; s[c].i = c; }
    qsort(s, (size_t)d, sizeof(orc_vi), orc_cmp_vi);
    int a = 0;
    while (a < d) {
        int b = a;
        while (b + 1 < d && s[b + 1].v == s[a].v) ++b;
        for (int k = a; k <= b; ++k) t[s[k].i] = a + b + 2;
        a = b + 1;
    }
    free(s);
}

/* Doubled midranks of one vector: counting for short vectors, sorting for long. */
void orc_rank2(const double* v, int d, int32_t* t) {
    if (d <= 64) orc_rank2_count(v, d, t);
    else orc_rank2_sort(v, d, t);
}

/* Doubled midranks of every row of an FP32 matrix given as doubles. */
void orc_rank2_rows(const double* V, int64_t rows, int d, int64_t ldv, int32_t* t, int64_t ldt) {
    for (int64_t r = 0; r < rows; ++r) orc_rank2(V + r * ldv, d, t + r * ldt);
}

/* --------------------------------------------- generalised Gini distance */

typedef struct {
    int d;
    double nu;
    double* g;     /* g[t] = Fbar^{nu-1} at doubled rank t, t = 0..2d (R2) */
    double g0;     /* Fbar(0)^{nu-1}, R(0) = (d+1)/2 */
    int32_t* t_pos;
    int32_t* t_neg;
    double* zneg;
} orc_gini_ws;

static void orc_ws_init(orc_gini_ws* w, int d, double nu) {
    w->d = d;
    w->nu = nu;
    w->g = (double*)malloc(sizeof(double) * (size_t)(2 * d + 1));
    for (int t = 0; t <= 2 * d; ++t) {
        double fbar = 1.0 - ((double)t / 2.0) / (double)d;   /* 1 - R/d */
        w->g[t] = pow(fbar, nu - 1.0);
    }
    w->g0 = pow(1.0 - ((double)(d + 1) / 2.0) / (double)d, nu - 1.0);
    w->t_pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)d);
    w->t_neg = (int32_t*)malloc(sizeof(int32_t) * (size_t)d);
    w->zneg = (double*)malloc(sizeof(double) * (size_t)d);
}

static void orc_ws_free(orc_gini_ws* w) {
    free(w->g); free(w->t_pos); free(w->t_neg); free(w->zneg);
}

/* Section III-B, asymmetric generalised Gini pseudo-distance written for the
 * difference z = x - y:  -d * sum_j z_j (Fbar(z_j)^{nu-1} - Fbar(0)^{nu-1}). */
static double orc_asym(const double* z, const int32_t* t, const orc_gini_ws* w) {
    double s = 0.0;
    for (int j = 0; j < w->d; ++j) s += z[j] * (w->g[t[j]] - w->g0);
    return -(double)w->d * s;
}

/* Section III-B, symmetrised distance: half D(x,y) plus half D(y,x).  D(y,x)
 * ranks y - x = -z afresh (no mirror identity is assumed).  Optional grad
 * returns d/dz_c with both rank vectors held fixed (R6):
 *   (d/2) (Fbar(-z_c)^{nu-1} - Fbar(z_c)^{nu-1}). */
static double orc_sym(const double* z, orc_gini_ws* w, double* grad) {
    const int d = w->d;
    for (int j = 0; j < d; ++j) w->zneg[j] = -z[j];
    orc_rank2(z, d, w->t_pos);
    orc_rank2(w->zneg, d, w->t_neg);
    double dxy = orc_asym(z, w->t_pos, w);
    double dyx = orc_asym(w->zneg, w->t_neg, w);
    if (grad) {
        for (int c = 0; c < d; ++c)
            grad[c] = 0.5 * (double)d * (w->g[w->t_neg[c]] - w->g[w->t_pos[c]]);
    }
    return 0.5 * dxy + 0.5 * dyx;
}

/* Generalised Gini pseudo-distance of a difference vector z (length d). */
double orc_gini_dist(const double* z, int d, double nu) {
    orc_gini_ws w;
    orc_ws_init(&w, d, nu);
    double r = orc_sym(z, &w, NULL);
    orc_ws_free(&w);
    return r;
}

/* Its rank-frozen gradient with respect to z; returns the distance. */
double orc_gini_dist_grad(const double* z, int d, double nu, double* grad) {
    orc_gini_ws w;
    orc_ws_init(&w, d, nu);
    double r = orc_sym(z, &w, grad);
    orc_ws_free(&w);
    return r;
}

/* Asymmetric form alone, for tests of the symmetrisation. */
double orc_gini_asym(const double* z, int d, double nu) {
    orc_gini_ws w;
    orc_ws_init(&w, d, nu);
    orc_rank2(z, d, w.t_pos);
    double r = orc_asym(z, w.t_pos, &w);
    orc_ws_free(&w);
    return r;
}

/* R8: coordinate difference as evaluated by the single-precision device. */
static double orc_diff(double a, double b, int mode) {
    if (mode == ORC_MATCH32) {
        float fa = (float)a;
        float fb = (float)b;
        float fz = fa - fb;
        return (double)fz;
    }
    return a - b;
}

/* Algorithm 1, distance-matrix step: the full symmetric n x n
 * matrix for each nu in the list (zero diagonal, pairs i<j computed, mirrored). */
void orc_dissim(const double* X, int64_t n, int m, int64_t ldx, int mode,
                const double* nus, int n_nu, double* Delta, int64_t ldd, int64_t stride_nu) {
    double* z = (double*)malloc(sizeof(double) * (size_t)m);
    for (int k = 0; k < n_nu; ++k) {
        orc_gini_ws w;
        orc_ws_init(&w, m, nus[k]);
        double* D = Delta + (int64_t)k * stride_nu;
        for (int64_t i = 0; i < n; ++i) {
            D[i * ldd + i] = 0.0;
            for (int64_t j = i + 1; j < n; ++j) {
                for (int c = 0; c < m; ++c) z[c] = orc_diff(X[i * ldx + c], X[j * ldx + c], mode);
                double v = orc_sym(z, &w, NULL);
                D[i * ldd + j] = v;
                D[j * ldd + i] = v;
            }
        }
        orc_ws_free(&w);
    }
    free(z);
}

/* The same distance for an explicit list of pairs (sampled checks at sizes
 * where the full matrix is out of reach). out[q*n_nu + k]. */
void orc_dissim_pairs(const double* X, int m, int64_t ldx, int mode, const int64_t* pi,
                      const int64_t* pj, int64_t npairs, const double* nus, int n_nu, double* out) {
    double* z = (double*)malloc(sizeof(double) * (size_t)m);
    for (int k = 0; k < n_nu; ++k) {
        orc_gini_ws w;
        orc_ws_init(&w, m, nus[k]);
        for (int64_t q = 0; q < npairs; ++q) {
            int64_t i = pi[q], j = pj[q];
            for (int c = 0; c < m; ++c) z[c] = orc_diff(X[i * ldx + c], X[j * ldx + c], mode);
            out[q * n_nu + k] = orc_sym(z, &w, NULL);
        }
        orc_ws_free(&w);
    }
    free(z);
}

/* Rounding scale of each dissimilarity, used by the tests' tolerances.  The
 * symmetrised distance is piecewise linear and homogeneous of degree one in z
 * (Section III-B), so with both rank vectors frozen D = sum_c z_c g_c, g its
 * gradient (orc_sym; Euler's identity).  S_ij = sum_c |z_c g_c| is the sum of
 * the absolute values of the terms whose sum is D_ij: S_ij >= |D_ij|, with
 * equality when no two terms differ in sign.  Full matrix, zero diagonal. */
void orc_dissim_scale(const double* X, int64_t n, int m, int64_t ldx, int mode, double nu,
                      double* S, int64_t lds) {
    double* z = (double*)malloc(sizeof(double) * (size_t)m);
    double* g = (double*)malloc(sizeof(double) * (size_t)m);
    orc_gini_ws w;
    orc_ws_init(&w, m, nu);
    for (int64_t i = 0; i < n; ++i) {
        S[i * lds + i] = 0.0;
        for (int64_t j = i + 1; j < n; ++j) {
            for (int c = 0; c < m; ++c) z[c] = orc_diff(X[i * ldx + c], X[j * ldx + c], mode);
            orc_sym(z, &w, g);
            double a = 0.0;
            for (int c = 0; c < m; ++c) a += fabs(z[c] * g[c]);
            S[i * lds + j] = a;
            S[j * lds + i] = a;
        }
    }
    orc_ws_free(&w);
    free(z); free(g);
}

/* ------------------------------------------------------------ the stress */

/* Latent distance and its gradient d delta / d u for u = Z_i - Z_j (R4, R6). */
static double orc_latent(const double* u, int p, int latent, orc_gini_ws* w, double* a) {
    if (latent == ORC_LATENT_GINI) return orc_sym(u, w, a);
    double s = 0.0;
    for (int c = 0; c < p; ++c) s += u[c] * u[c];
    double nrm = sqrt(s);
    for (int c = 0; c < p; ++c) a[c] = (nrm > 0.0) ? u[c] / nrm : 0.0;
    return nrm;
}

/* Raw stress (R5) sigma = sum_{i<j} (delta(Z_i - Z_j) - Delta_ij)^2 and its
 * gradient G (n x p, may be NULL): G_i += 2 r a, G_j -= 2 r a. */
/* Section IV-B, Kruskal stress KS = sqrt(sigma / sum_{i<j} Delta_ij^2): its
 * normaliser, summed over the pairs i < j. */
double orc_delta_sumsq(const double* Delta, int64_t n, int64_t ldd) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) s += Delta[i * ldd + j] * Delta[i * ldd + j];
    return s;
}

double orc_stress(const double* Delta, int64_t n, int64_t ldd, const double* Z, int p, int64_t ldz,
                  double nu, int latent, int mode, double* G, int64_t ldg) {
    orc_gini_ws w;
    orc_ws_init(&w, p, nu);
    double* u = (double*)malloc(sizeof(double) * (size_t)p);
    double* a = (double*)malloc(sizeof(double) * (size_t)p);
    if (G)
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < p; ++c) G[i * ldg + c] = 0.0;
    double sigma = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            for (int c = 0; c < p; ++c) u[c] = orc_diff(Z[i * ldz + c], Z[j * ldz + c], mode);
            double delta = orc_latent(u, p, latent, &w, a);
            double r = delta - Delta[i * ldd + j];
            sigma += r * r;
            if (G) {
                for (int c = 0; c < p; ++c) {
                    G[i * ldg + c] += 2.0 * r * a[c];
                    G[j * ldg + c] -= 2.0 * r * a[c];
                }
            }
        }
    }
    free(u); free(a);
    orc_ws_free(&w);
    return sigma;
}

/* Gradient rows for selected points only: G_i = sum_{j != i} 2 r_ij a(Z_i - Z_j),
 * reading row i of Delta from Drows[q*ldr + j]. Returns sum over the selected
 * rows of sum_{j>i} r_ij^2. */
double orc_grad_rows(const double* Drows, int64_t ldr, const int64_t* rows, int64_t nrows, int64_t n,
                     const double* Z, int p, int64_t ldz, double nu, int latent, int mode,
                     double* G, int64_t ldg) {
    orc_gini_ws w;
    orc_ws_init(&w, p, nu);
    double* u = (double*)malloc(sizeof(double) * (size_t)p);
    double* a = (double*)malloc(sizeof(double) * (size_t)p);
    double part = 0.0;
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t i = rows[q];
        for (int c = 0; c < p; ++c) G[q * ldg + c] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            for (int c = 0; c < p; ++c) u[c] = orc_diff(Z[i * ldz + c], Z[j * ldz + c], mode);
            double delta = orc_latent(u, p, latent, &w, a);
            double r = delta - Drows[q * ldr + j];
            if (j > i) part += r * r;
            for (int c = 0; c < p; ++c) G[q * ldg + c] += 2.0 * r * a[c];
        }
    }
    free(u); free(a);
    orc_ws_free(&w);
    return part;
}

/* Rounding scale of the gradient, used by the tests' tolerances: for each
 * selected point i and coordinate c, the sum over j != i of the absolute
 * values of the terms whose sum is G_ic -- |2 r_ij a_c| for the raw stress
 * (loss 0, as in orc_stress), |2 r_ij a_c| / (S Delta_ij) for Sammon's stress
 * (loss 1, as in orc_sammon, with S its normaliser passed by the caller and
 * no term for Delta_ij <= 0).  B_ic >= |G_ic|, with equality when the terms
 * of (i, c) share one sign.  Row i of Delta is read from Drows[q*ldr + j]. */
void orc_grad_scale_rows(const double* Drows, int64_t ldr, const int64_t* rows, int64_t nrows, int64_t n,
                         const double* Z, int p, int64_t ldz, double nu, int latent, int mode, int loss,
                         double S, double* B, int64_t ldb) {
    orc_gini_ws w;
    orc_ws_init(&w, p, nu);
    double* u = (double*)malloc(sizeof(double) * (size_t)p);
    double* a = (double*)malloc(sizeof(double) * (size_t)p);
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t i = rows[q];
        for (int c = 0; c < p; ++c) B[q * ldb + c] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double d = Drows[q * ldr + j];
            if (loss == 1 && !(d > 0.0)) continue;
            for (int c = 0; c < p; ++c) u[c] = orc_diff(Z[i * ldz + c], Z[j * ldz + c], mode);
            double delta = orc_latent(u, p, latent, &w, a);
            double r = delta - d;
            for (int c = 0; c < p; ++c) {
                double t = 2.0 * r * a[c];
                if (loss == 1) t = t / d / S;
                B[q * ldb + c] += fabs(t);
            }
        }
    }
    free(u); free(a);
    orc_ws_free(&w);
}

/* R7: default step for fixed-step gradient descent on the raw stress. */
double orc_step_size(int64_t n, int p, double nu, int latent) {
    double c = 1.0;
    if (latent == ORC_LATENT_GINI) {
        double* u = (double*)malloc(sizeof(double) * (size_t)p);
        double* a = (double*)malloc(sizeof(double) * (size_t)p);
        for (int k = 0; k < p; ++k) u[k] = (double)k;     /* any tie-free vector */
        orc_gini_dist_grad(u, p, nu, a);
        c = 0.0;
        for (int k = 0; k < p; ++k) c += a[k] * a[k];
        free(u); free(a);
    }
    return 1.0 / (2.0 * (double)n * c);
}

/* The MDS fit of Algorithm 1 read as R5-R7: iters fixed steps Z <- Z - eta G,
 * recording sigma(Z_t) before each step.  eta <= 0 selects the default. */
void orc_solve(const double* Delta, int64_t n, int64_t ldd, double* Z, int p, int64_t ldz, double nu,
               int latent, int mode, int iters, double eta, double* sigma_hist) {
    if (eta <= 0.0) eta = orc_step_size(n, p, nu, latent);
    double* G = (double*)malloc(sizeof(double) * (size_t)(n * p));
    for (int it = 0; it < iters; ++it) {
        double s = orc_stress(Delta, n, ldd, Z, p, ldz, nu, latent, mode, G, p);
        if (sigma_hist) sigma_hist[it] = s;
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < p; ++c) Z[i * ldz + c] -= eta * G[i * p + c];
    }
    free(G);
}

/* Section IV-B, Sammon's stress: with S = sum_{i<j} Delta_ij,
 *     (1/S) sum_{i<j} (delta_ij - Delta_ij)^2 / Delta_ij,
 * a pair with Delta_ij = 0 carrying no weight (its weight is undefined), and
 * its gradient with the latent ranks fixed. */
double orc_sammon(const double* Delta, int64_t n, int64_t ldd, const double* Z, int p, int64_t ldz, double nu,
                  int latent, int mode, double* G, int64_t ldg) {
    orc_gini_ws w;
    orc_ws_init(&w, p, nu);
    double* u = (double*)malloc(sizeof(double) * (size_t)p);
    double* a = (double*)malloc(sizeof(double) * (size_t)p);
    double S = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) S += Delta[i * ldd + j];
    if (G)
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < p; ++c) G[i * ldg + c] = 0.0;
    double sigma = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            const double d = Delta[i * ldd + j];
            if (!(d > 0.0)) continue;
            for (int c = 0; c < p; ++c) u[c] = orc_diff(Z[i * ldz + c], Z[j * ldz + c], mode);
            double delta = orc_latent(u, p, latent, &w, a);
            double r = delta - d;
            sigma += r * r / d;
            if (G) {
                for (int c = 0; c < p; ++c) {
                    G[i * ldg + c] += 2.0 * r / d * a[c];
                    G[j * ldg + c] -= 2.0 * r / d * a[c];
                }
            }
        }
    }
    if (G)
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < p; ++c) G[i * ldg + c] = S > 0.0 ? G[i * ldg + c] / S : 0.0;
    free(u); free(a);
    orc_ws_free(&w);
    return S > 0.0 ? sigma / S : 0.0;
}

/* A fixed step for the Sammon stress, 1 / (4 c max_i sum_{j != i} w_ij) with
 * w_ij = 1 / (S Delta_ij) and c as in orc_step_size: the weighted Laplacian's
 * largest eigenvalue is at most 2 max_i sum_j w_ij (Gershgorin), so the step
 * never leaves the majorising quadratic and the stress does not increase
 * (Euclidean latent distance, or the p = 2 Gini one). */
double orc_sammon_step(const double* Delta, int64_t n, int64_t ldd, int p, double nu, int latent) {
    double S = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) S += Delta[i * ldd + j];
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double d = (j > i) ? Delta[i * ldd + j] : Delta[j * ldd + i];
            if (j != i && d > 0.0) r += 1.0 / d;
        }
        if (r > mx) mx = r;
    }
    const double c = 1.0 / (2.0 * (double)n * orc_step_size(n, p, nu, latent));
    return (mx > 0.0) ? S / (4.0 * c * mx) : 0.0;
}

/* Fixed-step descent on the Sammon stress; eta <= 0 selects orc_sammon_step. */
void orc_solve_sammon(const double* Delta, int64_t n, int64_t ldd, double* Z, int p, int64_t ldz, double nu,
                      int latent, int mode, int iters, double eta, double* sigma_hist) {
    if (eta <= 0.0) eta = orc_sammon_step(Delta, n, ldd, p, nu, latent);
    double* G = (double*)malloc(sizeof(double) * (size_t)(n * p));
    for (int it = 0; it < iters; ++it) {
        double s = orc_sammon(Delta, n, ldd, Z, p, ldz, nu, latent, mode, G, p);
        if (sigma_hist) sigma_hist[it] = s;
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < p; ++c) Z[i * ldz + c] -= eta * G[i * p + c];
    }
    free(G);
}

