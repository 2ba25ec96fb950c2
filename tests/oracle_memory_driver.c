/* Memory and undefined-behaviour exercise of the C oracle, built with
 * AddressSanitizer and UBSan by tests/test_oracle_memory.py: ragged batches
 * with empty and one-atom clusters, both pair potentials, m = 0 and 10, and
 * basin hopping with a trace shorter than the run and a chain-index offset.
 * It checks no results (the other oracle tests do). */
#include "lj_oracle.c"
#include <stdio.h>
static uint64_t s_ = 88172645463325252ull;
static double urand(void) { s_ ^= s_ << 13; s_ ^= s_ >> 7; s_ ^= s_ << 17; return (s_ >> 11) * 0x1.0p-53; }
int main(void) {
    int32_t sizes[] = {0, 1, 2, 13, 38, 0, 100, 3};
    int num = 8; int32_t off[9]; off[0] = 0;
    for (int b = 0; b < num; ++b) off[b + 1] = off[b] + sizes[b];
    int64_t total = off[num];
    double* x = malloc(sizeof(double) * 3 * total);
    for (int b = 0; b < num; ++b) {
        double L = 1.2 * cbrt(sizes[b] > 0 ? sizes[b] : 1);
        for (int a = off[b]; a < off[b + 1]; ++a)
            for (int d = 0; d < 3; ++d) x[d * total + a] = L * (urand() - 0.5);
    }
    double *E = malloc(sizeof(double) * num), *g = malloc(sizeof(double) * 3 * total);
    double *ea = malloc(sizeof(double) * num), *ga = malloc(sizeof(double) * 3 * total);
    for (int pair = 0; pair < 2; ++pair) {
        lj_o_energy_grad_batch(num, off, total, x, E, g, pair, 6.0);
        lj_o_energy_grad_batch(num, off, total, x, E, NULL, pair, 6.0);
        lj_o_abs_sums_batch(num, off, total, x, ea, ga, pair, 6.0);
    }
    lj_o_lbfgs p = {10, 1e-6, 200, 0.2, 1e-4, 30, 1e-10, 0, 6.0};
    double *gn = malloc(sizeof(double) * num); int32_t *it = malloc(4 * num), *ev = malloc(4 * num), *st = malloc(4 * num);
    double* xm = malloc(sizeof(double) * 3 * total); memcpy(xm, x, sizeof(double) * 3 * total);
    lj_o_minimize_batch(num, off, total, xm, &p, E, gn, it, ev, st);
    p.pair = 1; memcpy(xm, x, sizeof(double) * 3 * total);
    lj_o_minimize_batch(num, off, total, xm, &p, E, gn, it, ev, st);
    p.pair = 0; p.m = 0; memcpy(xm, x, sizeof(double) * 3 * total);
    lj_o_minimize_batch(num, off, total, xm, &p, E, gn, it, ev, st);
    p.m = 10; memcpy(xm, x, sizeof(double) * 3 * total);
    lj_o_minimize_batch(num, off, total, xm, &p, E, gn, it, ev, st);
    /* basin hopping on the minimised batch, with a trace shorter than the run */
    lj_o_chain* ch = malloc(sizeof(lj_o_chain) * num);
    for (int b = 0; b < num; ++b) { ch[b].e_cur = E[b]; ch[b].step = 0.4; ch[b].win_accepts = 0; ch[b].step_index = 0; ch[b].e_best_seen = INFINITY; ch[b].e_best_acc = E[b]; }
    lj_o_bh bh = {num, 4, 0.8, 10, 0.5, 0.9, 12345};
    int cap = 3, steps = 5;
    double *t1 = malloc(sizeof(double) * num * cap * 4), *tc = malloc(sizeof(double) * num * cap * bh.cands);
    int8_t* ta = malloc(num * cap);
    lj_o_trace tr = {t1, ta, t1 + num * cap, t1 + 2 * num * cap, t1 + 3 * num * cap, t1, tc, cap};
    double* xb = malloc(sizeof(double) * 3 * total); memcpy(xb, xm, sizeof(double) * 3 * total);
    p.max_iter = 100;
    lj_o_bh_run(num, off, total, xm, xb, ch, &bh, &p, steps, &tr, 0);
    lj_o_bh_run(2, off + 3, total, xm, xb, ch + 3, &bh, &p, 2, NULL, 3);
    printf("done E0=%g st=%d\n", E[3], st[3]);
    free(x); free(E); free(g); free(ea); free(ga); free(gn); free(it); free(ev); free(st); free(xm); free(ch); free(t1); free(tc); free(ta); free(xb);
    return 0;
}
