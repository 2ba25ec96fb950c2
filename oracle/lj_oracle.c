/*
 * FP64 CPU oracle for the Lennard-Jones Basin Hopping hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product path (the
 * HIP library under paper_2510_25938_amd/csrc) shares no code with it.
 *
 * Everything here is plain, single-threaded, sequential FP64, built with
 * -ffp-contract=off so that the only fused multiply-adds are the explicit
 * fma() calls written below.  Paper references are to Carmona et al.,
 * "Revisiting and Accelerating the Basin Hopping Algorithm for Lennard-Jones
 * Clusters" (arXiv 2510.25938):
 *
 *   Eq. (1), Methodology / Lennard-Jones Potential   -> lj_o_energy_grad
 *   Methodology / Algorithm Overview, step 1          -> lj_o_perturb
 *   Methodology / Algorithm Overview, step 2          -> lj_o_minimize
 *   Methodology / Algorithm Overview, steps 3-5       -> lj_o_bh_decide
 *   Results, Figs. 2-3 (trial / accepted / lowest)    -> trace rows
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   - reduced units, sigma = epsilon = 1;
 *   - analytic gradient (the derivative of Eq. 1);
 *   - summation order: every per-atom sum runs over partner j in ascending
 *     order; sums over atoms use pairwise summation (Higham, "Accuracy and
 *     Stability of Numerical Algorithms", sec. 4.2) over the atom index padded
 *     with zeros to a power of two;
 *   - the paper's L-BFGS-B has no active bounds, so it is L-BFGS (Nocedal
 *     1980; Nocedal & Wright, "Numerical Optimization", Alg. 7.4) with m pairs,
 *     a per-atom step cap and a backtracking Armijo line search;
 *   - convergence on the Euclidean norm of the full 3N gradient;
 *   - perturbation draws, uniform on [-s, s) per coordinate, and the
 *     Metropolis draw come from Philox4x64-10 (Salmon et al., SC'11) keyed by
 *     (seed, chain, step, candidate), so they are order-free and resumable;
 *   - exp() in the Metropolis test is a fixed Cody-Waite + Taylor evaluation
 *     (exp_bh) so acceptance is reproducible bit for bit on any machine;
 *   - adaptation multiplies / divides the step size by a factor (0.9) every
 *     `interval` steps according to the windowed acceptance count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LJ_O_CONVERGED 0
#define LJ_O_MAXITER 1
#define LJ_O_LSFAIL 2
#define LJ_O_NONFINITE 3

/* ------------------------------------------------------------------------ */
/* Pairwise (tree) summation over v[0..n), zero-padded to a power of two.   */
/* ------------------------------------------------------------------------ */

static double tree_sum_pow2(const double* v, int64_t p) {
    if (p == 1) return v[0];
    return tree_sum_pow2(v, p / 2) + tree_sum_pow2(v + p / 2, p / 2);
}

static int64_t next_pow2(int64_t n) {
    int64_t p = 1;
    while (p < n) p *= 2;
    return p;
}

/* Sum of v[0..n) in pairwise order; v must have room for next_pow2(n)
 * entries; entries n.. are overwritten with zeros. */
static double tree_sum(double* v, int64_t n) {
    if (n <= 0) return 0.0;
    int64_t p = next_pow2(n);
    for (int64_t i = n; i < p; ++i) v[i] = 0.0;
    return tree_sum_pow2(v, p);
}

double lj_o_tree_sum(const double* v, int64_t n) {
    if (n <= 0) return 0.0;
    int64_t p = next_pow2(n);
    double* w = (double*)calloc((size_t)p, sizeof(double));
    memcpy(w, v, (size_t)n * sizeof(double));
    double s = tree_sum_pow2(w, p);
    free(w);
    return s;
}

double lj_o_exp_bh(double z);

/* Pair potentials: Eq. (1) (reduced units) or the Morse pair.              */
#define LJ_O_PAIR_LJ 0
#define LJ_O_PAIR_MORSE 1

/* ------------------------------------------------------------------------ */
/* Eq. (1): E = 4 sum_{i<j} (r^-12 - r^-6) and its analytic gradient.       */
/*                                                                          */
/* Written per atom over ordered pairs: E = 2 * sum_i e_i with               */
/* e_i = sum_{j != i} (r_ij^-12 - r_ij^-6).  With q = 1/r^2 and s6 = q^3,    */
/* dE/dx_i = sum_{j != i} q s6 (24 - 48 s6) (x_i - x_j).                     */
/* x, y, z point at the cluster's n coordinates; tmp has next_pow2(n) room. */
/* ------------------------------------------------------------------------ */
static double energy_grad_lj(int n, const double* x, const double* y, const double* z,
                             double* gx, double* gy, double* gz, double* tmp) {
    for (int i = 0; i < n; ++i) {
        double e = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j];
            double dy = y[i] - y[j];
            double dz = z[i] - z[j];
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            double q = 1.0 / r2;
            double s6 = (q * q) * q;
            e = e + fma(s6, s6, -s6);
            double f = (q * s6) * fma(-48.0, s6, 24.0);
            ax = fma(f, dx, ax);
            ay = fma(f, dy, ay);
            az = fma(f, dz, az);
        }
        tmp[i] = e;
        if (gx) {
            gx[i] = ax;
            gy[i] = ay;
            gz[i] = az;
        }
    }
    return 2.0 * tree_sum(tmp, n);
}

/* ------------------------------------------------------------------------ */
/* Morse pair (an empirical pair force field; the paper's conclusions name   */
/* empirical force fields as the next potentials), in reduced units with    */
/* well depth 1 at r = 1 and range rho:                                     */
/*   V(r) = t (t - 2),  t = exp(rho (1 - r)),  dV/dr = -2 rho t (t - 1).    */
/* Written per atom over ordered pairs: E = sum_{i<j} V = 0.5 sum_i e_i with */
/* e_i = sum_{j != i} V(r_ij), and dE/dx_i = sum_{j != i} (dV/dr / r)        */
/* (x_i - x_j).  r = IEEE sqrt(r^2); exp is exp_bh below (its reduction and  */
/* polynomial hold for any z <= 709; here z <= rho).                        */
/* ------------------------------------------------------------------------ */
static double energy_grad_morse(int n, const double* x, const double* y, const double* z,
                                double* gx, double* gy, double* gz, double* tmp, double rho) {
    const double c = -2.0 * rho;
    for (int i = 0; i < n; ++i) {
        double e = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j];
            double dy = y[i] - y[j];
            double dz = z[i] - z[j];
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            double r = sqrt(r2);
            double t = lj_o_exp_bh(fma(-rho, r, rho));
            e = e + t * (t - 2.0);
            double f = ((c * t) * (t - 1.0)) / r;
            ax = fma(f, dx, ax);
            ay = fma(f, dy, ay);
            az = fma(f, dz, az);
        }
        tmp[i] = e;
        if (gx) {
            gx[i] = ax;
            gy[i] = ay;
            gz[i] = az;
        }
    }
    return 0.5 * tree_sum(tmp, n);
}

static double energy_grad(int n, const double* x, const double* y, const double* z,
                          double* gx, double* gy, double* gz, double* tmp, int pair,
                          double rho) {
    if (pair == LJ_O_PAIR_MORSE) return energy_grad_morse(n, x, y, z, gx, gy, gz, tmp, rho);
    return energy_grad_lj(n, x, y, z, gx, gy, gz, tmp);
}

/* Sums of absolute pair terms, used by tests to bound the error of reduced
 * precision evaluations.  Eq. (1): eabs = 2 sum_i sum_{j!=i} (r^-12 + r^-6);
 * Morse: eabs = 0.5 sum_i sum_{j!=i} (t^2 + 2 t).  Per atom and component,
 * gabs = sum_{j!=i} |f_ij (x_i - x_j)|. */
static void abs_sums(int n, const double* x, const double* y, const double* z,
                     double* eabs, double* gax, double* gay, double* gaz, int pair,
                     double rho) {
    double tot = 0.0;
    for (int i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            double f;
            if (pair == LJ_O_PAIR_MORSE) {
                double r = sqrt(r2);
                double t = exp(rho * (1.0 - r));
                tot += t * t + 2.0 * t;
                f = 2.0 * rho * t * (t + 1.0) / r;
            } else {
                double q = 1.0 / r2;
                double s6 = q * q * q;
                tot += s6 * s6 + s6;
                f = fabs(q * s6 * (24.0 + 48.0 * s6));
            }
            ax += f * fabs(dx);
            ay += f * fabs(dy);
            az += f * fabs(dz);
        }
        gax[i] = ax;
        gay[i] = ay;
        gaz[i] = az;
    }
    *eabs = (pair == LJ_O_PAIR_MORSE ? 0.5 : 2.0) * tot;
}

/* Batched entry: xyz is three planes [3][total] (x plane, y plane, z plane);
 * cluster b owns atoms offset[b] .. offset[b+1]-1.  grad may be NULL. */
int lj_o_energy_grad_batch(int32_t num, const int32_t* offset, int64_t total,
                           const double* xyz, double* energy, double* grad, int32_t pair,
                           double rho) {
    int maxn = 0;
    for (int b = 0; b < num; ++b) {
        int n = offset[b + 1] - offset[b];
        if (n < 0) return -1;
        if (n > maxn) maxn = n;
    }
    double* tmp = (double*)malloc((size_t)next_pow2(maxn > 0 ? maxn : 1) * sizeof(double));
    for (int b = 0; b < num; ++b) {
        int64_t o = offset[b];
        int n = offset[b + 1] - offset[b];
        energy[b] = energy_grad(n, xyz + o, xyz + total + o, xyz + 2 * total + o,
                                grad ? grad + o : NULL, grad ? grad + total + o : NULL,
                                grad ? grad + 2 * total + o : NULL, tmp, pair, rho);
    }
    free(tmp);
    return 0;
}

int lj_o_abs_sums_batch(int32_t num, const int32_t* offset, int64_t total, const double* xyz,
                        double* eabs, double* gabs, int32_t pair, double rho) {
    for (int b = 0; b < num; ++b) {
        int64_t o = offset[b];
        int n = offset[b + 1] - offset[b];
        abs_sums(n, xyz + o, xyz + total + o, xyz + 2 * total + o, &eabs[b], gabs + o,
                 gabs + total + o, gabs + 2 * total + o, pair, rho);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* L-BFGS (the paper's L-BFGS-B with no active bounds).                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t m;           /* stored correction pairs                         */
    double gtol;         /* stop when ||g||_2 < gtol                        */
    int32_t max_iter;    /* accepted-step cap                               */
    double max_step;     /* per-atom displacement cap of the trial step     */
    double c1;           /* Armijo constant                                 */
    int32_t max_ls;      /* backtracking halvings per line search           */
    double curv_eps;     /* store (s,y) only if s.y > curv_eps |s| |y|      */
    int32_t pair;        /* LJ_O_PAIR_LJ (Eq. 1) or LJ_O_PAIR_MORSE         */
    double rho;          /* Morse range                                     */
} lj_o_lbfgs;

/* Relative energy change treated as rounding noise by the line search:
 * 4 ulps of |E| (2^-50). */
#define LJ_O_LS_RESOLUTION 0x1.0p-50

/* A 3N-vector of one cluster is held as three planes of n doubles. */
typedef struct {
    double* c[3];
} vec3n;

/* Dot product: per atom fma(az,bz, fma(ay,by, ax*bx)), then pairwise over atoms. */
static double dot3(int n, vec3n a, vec3n b, double* tmp) {
    for (int i = 0; i < n; ++i)
        tmp[i] = fma(a.c[2][i], b.c[2][i], fma(a.c[1][i], b.c[1][i], a.c[0][i] * b.c[0][i]));
    return tree_sum(tmp, n);
}

static vec3n vec_alloc(int n) {
    vec3n v;
    for (int k = 0; k < 3; ++k) v.c[k] = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    return v;
}
static void vec_free(vec3n v) {
    for (int k = 0; k < 3; ++k) free(v.c[k]);
}
static void vec_copy(int n, vec3n dst, vec3n src) {
    for (int k = 0; k < 3; ++k) memcpy(dst.c[k], src.c[k], (size_t)n * sizeof(double));
}

static double eval(int n, vec3n x, vec3n g, double* tmp, const lj_o_lbfgs* p) {
    return energy_grad(n, x.c[0], x.c[1], x.c[2], g.c[0], g.c[1], g.c[2], tmp, p->pair, p->rho);
}

/* Two-loop recursion (Nocedal & Wright, Alg. 7.4): r = H g, where H is the
 * L-BFGS inverse-Hessian approximation built from the `hist` stored pairs
 * (ring slots, newest at `newest`) on top of H0 = gamma I (H0 = I when no
 * pair is stored).  The search direction is d = -r. */
static void two_loop(int n, int m, int hist, int newest, const vec3n* S, const vec3n* Y,
                     const double* rho, double gamma, vec3n g, vec3n r, double* alpha_k,
                     double* tmp) {
    vec_copy(n, r, g);
    for (int t = 0; t < hist; ++t) { /* newest -> oldest */
        int k = ((newest - t) % m + m) % m;
        double a = rho[k] * dot3(n, S[k], r, tmp);
        alpha_k[k] = a;
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < n; ++i) r.c[c][i] = fma(-a, Y[k].c[c][i], r.c[c][i]);
    }
    if (hist > 0)
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < n; ++i) r.c[c][i] = gamma * r.c[c][i];
    for (int t = hist - 1; t >= 0; --t) { /* oldest -> newest */
        int k = ((newest - t) % m + m) % m;
        double b = rho[k] * dot3(n, Y[k], r, tmp);
        double w = alpha_k[k] - b;
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < n; ++i) r.c[c][i] = fma(w, S[k].c[c][i], r.c[c][i]);
    }
}

/* Exported for tests: S, Y are [hist][3][n] (oldest pair first), g and d are
 * [3][n]; writes the L-BFGS direction d = -H g. */
int lj_o_two_loop(int n, int hist, const double* S, const double* Y, const double* rho,
                  double gamma, const double* g, double* d) {
    int m = hist > 0 ? hist : 1;
    vec3n* Sv = (vec3n*)malloc(sizeof(vec3n) * (size_t)m);
    vec3n* Yv = (vec3n*)malloc(sizeof(vec3n) * (size_t)m);
    for (int k = 0; k < hist; ++k)
        for (int c = 0; c < 3; ++c) {
            Sv[k].c[c] = (double*)(S + ((size_t)k * 3 + (size_t)c) * (size_t)n);
            Yv[k].c[c] = (double*)(Y + ((size_t)k * 3 + (size_t)c) * (size_t)n);
        }
    vec3n gv, rv;
    for (int c = 0; c < 3; ++c) gv.c[c] = (double*)(g + (size_t)c * (size_t)n);
    rv = vec_alloc(n);
    double* alpha = (double*)calloc((size_t)m, sizeof(double));
    double* tmp = (double*)calloc((size_t)next_pow2(n > 0 ? n : 1), sizeof(double));
    two_loop(n, m, hist, hist - 1, Sv, Yv, rho, gamma, gv, rv, alpha, tmp);
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < n; ++i) d[(size_t)c * (size_t)n + (size_t)i] = -rv.c[c][i];
    vec_free(rv);
    free(alpha);
    free(tmp);
    free(Sv);
    free(Yv);
    return 0;
}

/*
 * Minimise one cluster in place.  x: three coordinate planes of n doubles.
 * Returns the status; E, gnorm, iters, evals receive the final values.
 *
 * Each iteration: test ||g||; two-loop recursion for d = -H g; restart from
 * -g if d is not a descent direction; cap the largest per-atom displacement
 * of d at max_step; backtrack alpha = 1, 1/2, 1/4, ... until the Armijo
 * condition E(x + alpha d) <= E + c1 alpha g.d holds; form s and y and store
 * them when the curvature s.y is positive enough.  A line search fails when
 * no trial passes, or when the accepted trial point equals x (s = 0: the
 * Armijo test cannot see a decrease below half an ulp of E, and a null step
 * makes no progress).  A failed line search with stored pairs discards the
 * pairs and retries from -g (not counted as an iteration); a failed line
 * search from -g ends the run (LSFAIL).
 */
static int minimize_one(int n, vec3n x, const lj_o_lbfgs* p, double* E_out, double* gnorm_out,
                        int32_t* iters_out, int32_t* evals_out) {
    const int m = p->m;
    double* tmp = (double*)calloc((size_t)next_pow2(n > 0 ? n : 1), sizeof(double));
    vec3n g = vec_alloc(n), d = vec_alloc(n), xt = vec_alloc(n), gt = vec_alloc(n);
    vec3n q = vec_alloc(n);
    vec3n* S = (vec3n*)malloc(sizeof(vec3n) * (size_t)(m > 0 ? m : 1));
    vec3n* Y = (vec3n*)malloc(sizeof(vec3n) * (size_t)(m > 0 ? m : 1));
    double* rho = (double*)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    double* alpha_k = (double*)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    for (int k = 0; k < m; ++k) {
        S[k] = vec_alloc(n);
        Y[k] = vec_alloc(n);
    }
    int hist = 0;   /* number of stored pairs                        */
    int newest = -1; /* ring slot of the newest pair                  */
    double gamma = 1.0;
    int32_t iters = 0, evals = 0;
    int status;
    double E = eval(n, x, g, tmp, p);
    ++evals;
    double gnorm = 0.0;
    const double ms2 = p->max_step * p->max_step;

    for (;;) {
        double gg = dot3(n, g, g, tmp);
        gnorm = sqrt(gg);
        if (!isfinite(E) || !isfinite(gg)) {
            status = LJ_O_NONFINITE;
            break;
        }
        if (gnorm < p->gtol) {
            status = LJ_O_CONVERGED;
            break;
        }
        if (iters >= p->max_iter) {
            status = LJ_O_MAXITER;
            break;
        }

        two_loop(n, m, hist, newest, S, Y, rho, gamma, g, q, alpha_k, tmp);
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < n; ++i) d.c[c][i] = -q.c[c][i];

        double gd = dot3(n, g, d, tmp);
        if (hist > 0 && !(gd < 0.0)) { /* not a descent direction: restart */
            hist = 0;
            for (int c = 0; c < 3; ++c)
                for (int i = 0; i < n; ++i) d.c[c][i] = -g.c[c][i];
            gd = dot3(n, g, d, tmp);
        }

        /* Per-atom step cap. */
        double dmax2 = 0.0;
        for (int i = 0; i < n; ++i) {
            double a2 = fma(d.c[2][i], d.c[2][i], fma(d.c[1][i], d.c[1][i], d.c[0][i] * d.c[0][i]));
            if (a2 > dmax2) dmax2 = a2;
        }
        if (dmax2 > ms2) {
            double sc = p->max_step / sqrt(dmax2);
            for (int c = 0; c < 3; ++c)
                for (int i = 0; i < n; ++i) d.c[c][i] = d.c[c][i] * sc;
            gd = dot3(n, g, d, tmp);
        }

        /* Backtracking Armijo line search.  When E_t and E differ by no more
         * than LJ_O_LS_RESOLUTION |E| (4 ulps of E) the energy test is decided
         * by the rounding of the energy sums; the trial is then judged by the
         * derivative form of sufficient decrease (the approximate Armijo
         * condition of Hager & Zhang, 2005: with the trapezoidal estimate
         * E_t - E ~ alpha (g.d + g_t.d) / 2, E_t - E <= c1 alpha g.d becomes
         * g_t.d <= (2 c1 - 1) g.d), which the gradients resolve. */
        double alpha = 1.0, Et = 0.0;
        int ok = 0;
        for (int ls = 0; ls < p->max_ls; ++ls) {
            for (int c = 0; c < 3; ++c)
                for (int i = 0; i < n; ++i) xt.c[c][i] = fma(alpha, d.c[c][i], x.c[c][i]);
            Et = eval(n, xt, gt, tmp, p);
            ++evals;
            if (Et <= fma(p->c1 * alpha, gd, E)) {
                ok = 1;
                break;
            }
            if (fabs(Et - E) <= LJ_O_LS_RESOLUTION * fabs(E) &&
                dot3(n, gt, d, tmp) <= (2.0 * p->c1 - 1.0) * gd) {
                ok = 1;
                break;
            }
            alpha = alpha * 0.5;
        }
        if (!ok) {
            if (hist > 0) {
                hist = 0;
                continue;
            }
            status = LJ_O_LSFAIL;
            break;
        }

        /* Curvature pair. s = x_t - x, y = g_t - g (x, g are overwritten below). */
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < n; ++i) {
                d.c[c][i] = xt.c[c][i] - x.c[c][i]; /* d now holds s */
                q.c[c][i] = gt.c[c][i] - g.c[c][i]; /* q now holds y */
            }
        double sy = dot3(n, d, q, tmp);
        double yy = dot3(n, q, q, tmp);
        double ss = dot3(n, d, d, tmp);
        if (ss == 0.0) {
            /* The accepted trial point equals x in every coordinate (alpha d is
             * below the coordinates' resolution): no progress is possible along
             * d, so this counts as a failed line search. */
            if (hist > 0) {
                hist = 0;
                continue;
            }
            status = LJ_O_LSFAIL;
            break;
        }
        if (m > 0 && sy > p->curv_eps * sqrt(ss * yy)) {
            newest = (newest + 1) % m;
            vec_copy(n, S[newest], d);
            vec_copy(n, Y[newest], q);
            rho[newest] = 1.0 / sy;
            gamma = sy / yy;
            if (hist < m) ++hist;
        }
        vec_copy(n, x, xt);
        vec_copy(n, g, gt);
        E = Et;
        ++iters;
    }

    *E_out = E;
    *gnorm_out = gnorm;
    *iters_out = iters;
    *evals_out = evals;
    for (int k = 0; k < m; ++k) {
        vec_free(S[k]);
        vec_free(Y[k]);
    }
    free(S);
    free(Y);
    free(rho);
    free(alpha_k);
    vec_free(g);
    vec_free(d);
    vec_free(xt);
    vec_free(gt);
    vec_free(q);
    free(tmp);
    return status;
}

/* Batched local minimisation on SoA planes [3][total]; xyz is updated in place. */
int lj_o_minimize_batch(int32_t num, const int32_t* offset, int64_t total, double* xyz,
                        const lj_o_lbfgs* p, double* energy, double* gnorm, int32_t* iters,
                        int32_t* evals, int32_t* status) {
    for (int b = 0; b < num; ++b) {
        int64_t o = offset[b];
        int n = offset[b + 1] - offset[b];
        vec3n x;
        x.c[0] = xyz + o;
        x.c[1] = xyz + total + o;
        x.c[2] = xyz + 2 * total + o;
        status[b] = minimize_one(n, x, p, &energy[b], &gnorm[b], &iters[b], &evals[b]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the      */
/* published round function: two 64x64->128 multiplies per round, the key   */
/* bumped by the Weyl constants between rounds.                             */
/* ------------------------------------------------------------------------ */
void lj_o_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* 53 high bits of a word as a double in [0, 1). */
static double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

#define PURPOSE_PERTURB 3ULL
#define PURPOSE_METROPOLIS 4ULL

/* Random word number `word` (0-based) of the stream (seed; chain, step, purpose, cand). */
static uint64_t stream_word(uint64_t seed, uint64_t chain, uint64_t step, uint64_t purpose,
                            uint64_t cand, uint64_t word) {
    uint64_t ctr[4] = {word / 4, chain, step, (purpose << 32) | cand};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    lj_o_philox4x64_10(ctr, key, out);
    return out[word % 4];
}

/* ------------------------------------------------------------------------ */
/* exp_bh: exp(z) for the Metropolis test.  Cody & Waite (1980) reduction   */
/* z = k ln2 + r with ln2 split into a high part (32 significant bits, 21   */
/* trailing zero bits: k ln2_hi is exact for |k| < 2^21) and a low part;    */
/* the split is the published one of fdlibm's e_exp.c (Sun, 1993).  Then    */
/* the Taylor series of e^r to degree 13 in Horner form                     */
/* (|r| <= ln2/2, truncation below 2^-53), then scaling by 2^k.  Returns 0  */
/* for z < -708 or NaN.  The Metropolis test uses z <= 0; the Morse pair     */
/* uses z <= rho (the reduction and polynomial hold up to z = 709).         */
/* ------------------------------------------------------------------------ */
double lj_o_exp_bh(double z) {
    if (!(z >= -708.0)) return 0.0;
    const double log2e = 1.4426950408889634;        /* 1/ln 2 */
    const double ln2_hi = 6.93147180369123816490e-01; /* 0x3FE62E42FEE00000 */
    const double ln2_lo = 1.90821492927058770002e-10; /* 0x3DEA39EF35793C76 */
    double kf = rint(z * log2e);
    double r = fma(-kf, ln2_hi, z);
    r = fma(-kf, ln2_lo, r);
    double p = 1.0 / 6227020800.0; /* 1/13! */
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)kf);
}

/* ------------------------------------------------------------------------ */
/* Basin hopping (Algorithm Overview, steps 1-5).                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t chains;         /* independent chains                       */
    int32_t cands;          /* n candidates per step                    */
    double kT;              /* Metropolis temperature                   */
    int32_t adapt_interval; /* adapt every this many steps              */
    double target_rate;     /* target acceptance rate                   */
    double factor;          /* step multiplied / divided by this        */
    uint64_t seed;
} lj_o_bh;

/* Step 1: candidate `cand` of chain `chain` at step `step`: every coordinate
 * (flattened index k = 3*atom + dim, the paper's 1-D layout) is displaced by
 * s * (2u - 1), u uniform in [0,1), i.e. uniformly within a cube of side 2s. */
void lj_o_perturb(int n, const double* xcur /* planes [3][n] */, double s, uint64_t seed,
                  int64_t chain, int64_t step, int64_t cand, double* xc /* planes [3][n] */) {
    for (int a = 0; a < n; ++a)
        for (int dim = 0; dim < 3; ++dim) {
            uint64_t w = stream_word(seed, (uint64_t)chain, (uint64_t)step, PURPOSE_PERTURB,
                                     (uint64_t)cand, (uint64_t)(3 * a + dim));
            double v = 2.0 * u01(w) - 1.0;
            xc[dim * n + a] = fma(s, v, xcur[dim * n + a]);
        }
}

/* Per-chain state of the Markov chain (host copy). */
typedef struct {
    double e_cur;
    double step;
    int32_t win_accepts;
    int64_t step_index;
    double e_best_seen; /* lowest selected trial energy so far (Fig. 2, green)   */
    double e_best_acc;  /* lowest accepted energy so far (Fig. 3)                */
} lj_o_chain;

/* Steps 3-5 for one chain: select the lowest of the n candidate energies
 * (first index on ties, non-finite never selected), apply the Metropolis test,
 * update the bookkeeping and adapt the step size.  Returns the selected
 * candidate (-1 if none is finite); *accepted receives the decision. */
int lj_o_bh_decide(lj_o_chain* st, const lj_o_bh* p, int64_t chain, const double* ecand,
                   int32_t* accepted, int32_t* improved, double* e_sel) {
    int sel = -1;
    double best = INFINITY;
    for (int j = 0; j < p->cands; ++j)
        if (ecand[j] < best) {
            best = ecand[j];
            sel = j;
        }
    int acc = 0, imp = 0;
    if (sel >= 0) {
        double dE = best - st->e_cur;
        if (dE <= 0.0) {
            acc = 1;
        } else {
            uint64_t w = stream_word(p->seed, (uint64_t)chain, (uint64_t)st->step_index,
                                     PURPOSE_METROPOLIS, 0, 0);
            if (u01(w) < lj_o_exp_bh(-dE / p->kT)) acc = 1;
        }
        if (best < st->e_best_seen) st->e_best_seen = best;
        if (acc) {
            st->e_cur = best;
            st->win_accepts += 1;
            if (best < st->e_best_acc) {
                st->e_best_acc = best;
                imp = 1;
            }
        }
    }
    st->step_index += 1;
    if (st->step_index % p->adapt_interval == 0) {
        double target = p->target_rate * (double)p->adapt_interval;
        if ((double)st->win_accepts > target)
            st->step = st->step / p->factor;
        else if ((double)st->win_accepts < target)
            st->step = st->step * p->factor;
        st->win_accepts = 0;
    }
    *accepted = acc;
    *improved = imp;
    *e_sel = sel >= 0 ? best : NAN;
    return sel;
}

/* Per-step trace rows, each array [chains][cap] (ecand: [chains][cap][cands]);
 * any pointer may be NULL.  Row k holds the values after step k (0-based). */
typedef struct {
    double* e_trial;    /* selected candidate energy (NaN if none finite) */
    int8_t* accepted;   /* Metropolis decision                            */
    double* e_best;     /* lowest selected energy so far                  */
    double* e_best_acc; /* lowest accepted energy so far                  */
    double* e_cur;      /* current energy after the step                  */
    double* step;       /* step size after the step's adaptation          */
    double* ecand;      /* every candidate's final energy                 */
    int32_t cap;
} lj_o_trace;

/*
 * Full FP64 basin-hopping run of `num_steps` steps for every chain.
 * chain c owns atoms coff[c] .. coff[c+1]-1 of the SoA planes xcur/xbest
 * ([3][total]); its state is st[c]; xcur must hold a local minimum on entry.
 * Its random streams are those of chain chain0 + c, so a contiguous slice of
 * a larger set of chains can be run on its own with chain0 = its first index.
 */
int lj_o_bh_run(int32_t chains, const int32_t* coff, int64_t total, double* xcur, double* xbest,
                lj_o_chain* st, const lj_o_bh* p, const lj_o_lbfgs* lp, int32_t num_steps,
                const lj_o_trace* tr, int32_t chain0) {
    int32_t cap = tr ? tr->cap : 0;
    int maxn = 1;
    for (int c = 0; c < chains; ++c)
        if (coff[c + 1] - coff[c] > maxn) maxn = coff[c + 1] - coff[c];
    int nc = p->cands;
    double* cur = (double*)malloc(sizeof(double) * 3 * (size_t)maxn);
    double* cand = (double*)malloc(sizeof(double) * 3 * (size_t)maxn * (size_t)nc);
    double* ec = (double*)malloc(sizeof(double) * (size_t)nc);
    for (int c = 0; c < chains; ++c) {
        int n = coff[c + 1] - coff[c];
        int64_t o = coff[c];
        for (int dim = 0; dim < 3; ++dim)
            memcpy(cur + dim * n, xcur + dim * total + o, sizeof(double) * (size_t)n);
        for (int s = 0; s < num_steps; ++s) {
            int64_t k = st[c].step_index;
            for (int j = 0; j < nc; ++j) {
                double* xc = cand + (size_t)j * 3 * n;
                lj_o_perturb(n, cur, st[c].step, p->seed, chain0 + c, k, j, xc);
                vec3n v;
                v.c[0] = xc;
                v.c[1] = xc + n;
                v.c[2] = xc + 2 * n;
                double gn;
                int32_t it, ev;
                minimize_one(n, v, lp, &ec[j], &gn, &it, &ev);
            }
            int32_t acc, imp;
            double esel;
            int sel = lj_o_bh_decide(&st[c], p, chain0 + c, ec, &acc, &imp, &esel);
            if (acc) memcpy(cur, cand + (size_t)sel * 3 * n, sizeof(double) * 3 * (size_t)n);
            if (imp && xbest)
                for (int dim = 0; dim < 3; ++dim)
                    memcpy(xbest + dim * total + o, cur + dim * n, sizeof(double) * (size_t)n);
            if (k >= 0 && k < cap) {
                size_t r = (size_t)c * (size_t)cap + (size_t)k;
                if (tr->e_trial) tr->e_trial[r] = esel;
                if (tr->accepted) tr->accepted[r] = (int8_t)acc;
                if (tr->e_best) tr->e_best[r] = st[c].e_best_seen;
                if (tr->e_best_acc) tr->e_best_acc[r] = st[c].e_best_acc;
                if (tr->e_cur) tr->e_cur[r] = st[c].e_cur;
                if (tr->step) tr->step[r] = st[c].step;
                if (tr->ecand)
                    for (int j = 0; j < nc; ++j) tr->ecand[r * (size_t)nc + (size_t)j] = ec[j];
            }
        }
        for (int dim = 0; dim < 3; ++dim)
            memcpy(xcur + dim * total + o, cur + dim * n, sizeof(double) * (size_t)n);
    }
    free(cur);
    free(cand);
    free(ec);
    return 0;
}
