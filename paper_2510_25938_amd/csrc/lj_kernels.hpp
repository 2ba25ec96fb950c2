// Kernels of liblj_bh.so: batched energy+gradient, the persistent L-BFGS
// minimiser, and the basin-hopping perturb / decide / finalize kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lj_bh.h"
#include "lj_device.hpp"

namespace lj {

constexpr int kNumClasses = 4;        // cluster-size classes of the minimiser
constexpr int kClassMaxN[kNumClasses] = {64, 128, 256, LJ_MAX_ATOMS_MIN};
constexpr int kStatusBadSize = LJ_BADSIZE;

struct LbfgsDev {
    int m;
    double gtol;
    int max_iter;
    double max_step;
    double c1;
    int max_ls;
    double curv_eps;
    double gtol_mixed_per_atom;
    int polish;
    double ls_noise;
};

// Work list built by plan_kernel: candidate indices sorted by N descending,
// split into size classes (largest class first).
struct Plan {
    int32_t* list;      // [num]
    int32_t* cls;       // start[kNumClasses], count[kNumClasses]
    int32_t* queue;     // claim counters [kNumClasses]
};

// Units of the caller's coordinates and energies (lj_batch.sigma, .epsilon):
// the kernels work in reduced units, x_reduced = x / sigma, and report
// E = epsilon E_reduced and g = (epsilon / sigma) g_reduced.
struct Units {
    double sigma;
    double escale;  // epsilon
    double gscale;  // epsilon / sigma
    int scaled;     // sigma != 1
};

struct MinArgs {
    const int32_t* offset;
    int64_t total;
    double* xyz;
    double* energy;
    double* gnorm;
    int32_t* iters;
    int32_t* evals;
    int32_t* status;
    double* xyz_switch;
    Plan plan;
    int cls;
    double* hist;       // global history (class 3): per persistent workgroup
    LbfgsDev p;
    int pot;            // LJ_PAIR_LJ or LJ_PAIR_MORSE
    double rho;         // Morse range
    Units u;
    int max_n;          // the batch's largest cluster
    int up_n;           // set by launch_minimize_class (class_up_n)
};

// Launchers (lj_minimize.hip, lj_bh_kernels.hip).
struct EvalShape {
    int W, A;  // wavefronts per workgroup, atom slots per lane
};
constexpr int kNumLargeShapes = 3;  // minimiser shapes for N in 257..1024
EvalShape eval_shape(int max_n);
bool eval_shape_supported(EvalShape s);
hipError_t launch_energy_grad(int mixed, int pot, EvalShape s, int num, const int32_t* off,
                              int64_t total, const double* xyz, double* e, double* g, double rho,
                              Units u, hipStream_t st);
// Minimiser shapes per size class (see lj_minimize.hip): class_shapes(c)
// interchangeable kernels; shape s holds clusters of at most
// shape_max_n(c, s) atoms, shape_clusters_per_wg(c, s) of them per workgroup.
int class_of(int n);
int class_shapes(int c);
int shape_max_n(int c, int shape);
int shape_clusters_per_wg(int c, int shape);
int class_block(int c, int shape);
// Largest N that the unique-pair FP64 evaluation (Morse pair) serves in a
// launch of this shape on a batch of at most max_n atoms (0: none), and the
// dynamic LDS it takes (an up_n x up_n matrix of double2 and the list of the
// pairs).
constexpr int kUpMaxN = 40;
int class_up_n(int c, int shape, int max_n, int pot);
size_t class_dyn_lds(int c, int shape, int max_n, int pot);
size_t class_hist_bytes_per_wg(int c, int shape);
const void* minimize_kernel_for(int mixed, int pot, int c, int shape);
hipError_t launch_plan(const int32_t* offset, int num, int max_n, const int32_t* active, Plan plan,
                       int32_t* status, hipStream_t st);
hipError_t launch_minimize_class(int mixed, int c, int shape, int grid, const MinArgs& a,
                                 hipStream_t st);

struct BhDev {
    int cands;
    double kT;
    int adapt_interval;
    double target_rate;
    double factor;
    uint64_t seed;
};

struct BhStateDev {
    double* xyz_cur;
    double* e_cur;
    double* step;
    int32_t* win_accepts;
    int64_t* step_index;
    double* e_best_seen;
    double* e_best_acc;
    double* xyz_best;
};

struct BhTraceDev {
    double* e_trial;
    int8_t* accepted;
    double* e_best;
    double* e_best_acc;
    double* e_cur;
    double* step;
    double* e_cand;
    int8_t* polish_status;
    int32_t cap;
};

hipError_t launch_perturb(const int32_t* coff, int chains, int max_n, int64_t total_chain,
                          BhStateDev s, BhDev p, double* xc, int32_t* cand_off, hipStream_t st);
// fin != nullptr: no polish follows, so the same launch also does the step's
// final bookkeeping (trace row fin) and finalize is not launched.
hipError_t launch_decide(const int32_t* coff, int chains, int max_n, int64_t total_chain,
                         BhStateDev s, BhDev p, const double* xc, const double* ecand,
                         int32_t* dec, const BhTraceDev* fin, hipStream_t st);
hipError_t launch_finalize(const int32_t* coff, int chains, int max_n, int64_t total_chain,
                           BhStateDev s, BhDev p, const double* ecand, const int32_t* dec,
                           const double* polish_e, const int32_t* polish_st, BhTraceDev tr,
                           hipStream_t st);

}  // namespace lj
