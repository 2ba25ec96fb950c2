// Batched energy+gradient and the persistent L-BFGS minimiser (gfx950).
//
// Energy: Eq. (1) of Carmona et al.; minimiser: the paper's L-BFGS-B with no
// active bounds, i.e. L-BFGS (two-loop recursion of Nocedal & Wright,
// Alg. 7.4) with a per-atom step cap and a backtracking Armijo line search
// (Algorithm Overview, step 2).
//
// One workgroup ("team", W wavefronts) owns one cluster at a time and runs
// its whole minimisation on chip: coordinates are staged in LDS for the pair
// loop, all reductions go through wavefront butterflies and (for W > 1) a
// small LDS exchange, and for N <= 256 the m (s, y) history pairs stay in
// registers.  Teams are persistent: they claim clusters from a queue that
// lists the batch by N descending (longest first), one launch per size class
// (the size classes run concurrently on side streams).
#include <hip/hip_runtime.h>

#include "lj_kernels.hpp"

namespace lj {

// ---------------------------------------------------------------------------
// Team: LDS buffers and the collective operations of one workgroup, or (G > 1)
// of one of the G clusters packed in a one-wavefront workgroup, each on its
// own 64 / G lanes.  A packed team's values are uniform over its lanes only,
// so its reductions stay within those lanes and nothing is read out as a
// wavefront-uniform scalar; LDS order within one wavefront needs no barrier
// (a wavefront's LDS instructions execute in issue order).
// ---------------------------------------------------------------------------
// UP (Morse pair): the FP64 evaluation takes the unique-pair form
// (pairs_morse64_up) for clusters of at most up_n atoms, with an up_n x up_n
// pair matrix at upm.
template <int W, int A, int POT, int L = kWave, int G = 1, bool UP = false>
struct Team {
    static_assert(G == 1 || (W == 1 && A == 1 && L == kWave), "packing: one wavefront, one slot");
    static_assert(!UP || (W == 1 && A == 1 && G == 1 && POT == kPairMorse),
                  "unique pairs: Morse pair, one wavefront, one cluster");
    static constexpr int T = kWave * W;
    static constexpr int NVMAX = 4 * A;
    static constexpr int kG = G;
    double4* pos64;  // this team's atoms (a packed team: its own part of the buffer)
    float4* pos32;
    float* rbuf;  // reaction buffers of the FP32 tiles and the one-wavefront ring
    TeamScratch<W, NVMAX>* sc;
    int bank;
    int n;
    int li;      // atom index of this thread's slot 0 within the cluster
    double rho;  // Morse range (POT == kPairMorse)
    double2* upm;    // up_n x up_n pair matrix
    uint2* uplist;   // up_n (up_n - 1) / 2 pair-list entries
    int up_n;

    // Before the first evaluation of a cluster (n set): its pair list.
    __device__ __forceinline__ void prepare() {
        if constexpr (UP) {
            if (n <= up_n) {
                up_pair_list(n, uplist, li);
                __syncthreads();
            }
        }
    }

    __device__ __forceinline__ bool active(int a) const { return a * T + li < n; }

    // a value uniform over the team, as the team's scalar
    __device__ __forceinline__ int uni(int v) const {
        if constexpr (G > 1)
            return v;
        else
            return uniform(v);
    }

    __device__ __forceinline__ void sync() const {
        if constexpr (G > 1) {
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_wave_barrier();
        } else {
            __syncthreads();
        }
    }

    __device__ __forceinline__ double dot(const double (&u)[3][A], const double (&v)[3][A]) {
        double p[1][A], o[1];
#pragma unroll
        for (int a = 0; a < A; ++a) p[0][a] = fma(u[2][a], v[2][a], fma(u[1][a], v[1][a], u[0][a] * v[0][a]));
        if constexpr (G > 1) return group_sum<G>(p[0][0]);
        team_sum<W, A, 1, NVMAX, L>(p, o, *sc, bank);
        return o[0];
    }

    // (s.y, y.y, s.s, w.w) in one reduction.
    __device__ __forceinline__ void dot4(const double (&s)[3][A], const double (&y)[3][A],
                                         const double (&w)[3][A], double& sy, double& yy,
                                         double& ss, double& ww) {
        double p[4][A], o[4];
#pragma unroll
        for (int a = 0; a < A; ++a) {
            p[0][a] = fma(s[2][a], y[2][a], fma(s[1][a], y[1][a], s[0][a] * y[0][a]));
            p[1][a] = fma(y[2][a], y[2][a], fma(y[1][a], y[1][a], y[0][a] * y[0][a]));
            p[2][a] = fma(s[2][a], s[2][a], fma(s[1][a], s[1][a], s[0][a] * s[0][a]));
            p[3][a] = fma(w[2][a], w[2][a], fma(w[1][a], w[1][a], w[0][a] * w[0][a]));
        }
        if constexpr (G > 1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = group_sum<G>(p[k][0]);
        } else {
            team_sum<W, A, 4, NVMAX, L>(p, o, *sc, bank);
        }
        sy = o[0];
        yy = o[1];
        ss = o[2];
        ww = o[3];
    }

    // Largest per-atom squared norm of v.
    __device__ __forceinline__ double max_atom_norm2(const double (&v)[3][A]) {
        double m[A];
#pragma unroll
        for (int a = 0; a < A; ++a) m[a] = fma(v[2][a], v[2][a], fma(v[1][a], v[1][a], v[0][a] * v[0][a]));
        if constexpr (G > 1) return group_max<G>(m[0]);
        return team_max<W, A, NVMAX, L>(m, *sc, bank);
    }

    // u.v and the largest per-atom squared norm of v, with the same values as
    // dot() and max_atom_norm2() but one exchange between the wavefronts.
    // vmax2 is exact whenever it exceeds cap2; otherwise it is some value
    // <= cap2 (one wavefront: a ballot over the lanes skips the max when no
    // atom exceeds cap2).
    __device__ __forceinline__ void dot_max(const double (&u)[3][A], const double (&v)[3][A],
                                            double& uv, double& vmax2, double cap2) {
        double p[A], m = 0.0;
        double ws[A];
#pragma unroll
        for (int a = 0; a < A; ++a) {
            p[a] = fma(u[2][a], v[2][a], fma(u[1][a], v[1][a], u[0][a] * v[0][a]));
            const double n2 = fma(v[2][a], v[2][a], fma(v[1][a], v[1][a], v[0][a] * v[0][a]));
            m = a == 0 ? n2 : fmax(m, n2);
        }
        if constexpr (G > 1) {
            // a packed team: any value <= cap2 serves when no atom of the
            // wavefront exceeds cap2
            uv = group_sum<G>(p[0]);
            vmax2 = __builtin_amdgcn_ballot_w64(m > cap2) != 0 ? group_max<G>(m) : 0.0;
            return;
        }
#pragma unroll
        for (int a = 0; a < A; ++a) ws[a] = wave_sum<L>(p[a]);
        if constexpr (W == 1) {
            uv = tree<A>(ws);
            vmax2 = __builtin_amdgcn_ballot_w64(m > cap2) != 0 ? wave_max<L>(m) : 0.0;
        } else {
            m = wave_max<L>(m);
            const int w = threadIdx.x / kWave;
            if (threadIdx.x % kWave == 0) {
#pragma unroll
                for (int a = 0; a < A; ++a) sc->v[bank][a][w] = ws[a];
                sc->v[bank][A][w] = m;
            }
            __syncthreads();
            double r[A];
#pragma unroll
            for (int a = 0; a < A; ++a) {
                double rw[W];
#pragma unroll
                for (int q = 0; q < W; ++q) rw[q] = sc->v[bank][a][q];
                r[a] = tree_w<W>(rw);
            }
            double mx = sc->v[bank][A][0];
#pragma unroll
            for (int q = 1; q < W; ++q) mx = fmax(mx, sc->v[bank][A][q]);
            bank ^= 1;
            uv = uniform(tree<A>(r));
            vmax2 = uniform(mx);
        }
    }

    // E and g at x.  FP64: the ordered-pair loop in the oracle's order.
    // F32: FP32 pair arithmetic and per-atom FP32 partial sums, FP64 totals;
    // the unique-pair ring for one-wavefront clusters of 20 to 43 atoms, the
    // unique-pair 64-atom tiles above 32 atoms otherwise (Eq. (1)), else the
    // ordered loop.  Every loop reports e_i in the ordered-pair convention,
    // which counts each pair twice: E = 2 sum_i e_i for Eq. (1) (e_i holds
    // r^-12 - r^-6, a quarter of the pair energy) and E = 0.5 sum_i e_i for
    // the Morse pair (e_i holds V).
    template <bool F32>
    __device__ __forceinline__ double eval(const double (&x)[3][A], double (&g)[3][A]) {
        constexpr bool kTiles = F32 && POT == kPairLJ && kUseTiles<W, A> && G == 1;
        constexpr bool kRing = F32 && W == 1 && A == 1 && G == 1;
        bool ring = false, tiles = false;
        if constexpr (kRing) ring = ring_for(n);
        if constexpr (kTiles) tiles = !ring && tiles_for(n);
        sync();  // previous readers of the position and reaction buffers are done
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const int i = a * T + li;
            if (ring) {  // ring layout: pos[j] = atom j mod n for j < 64 + steps
                if (i < n) {
                    const float4 p = make_float4((float)x[0][a], (float)x[1][a], (float)x[2][a],
                                                 0.0f);
                    const int end = kWave + ring_steps(n);
                    for (int j = i; j < end; j += n) pos32[j] = p;
                }
            } else if (tiles) {  // tile layout: each 64-atom tile twice, padded
                if (i < ((n + kWave - 1) / kWave) * kWave) {
                    const float4 p = i < n ? make_float4((float)x[0][a], (float)x[1][a],
                                                         (float)x[2][a], 0.0f)
                                           : tile_pad(i);
                    pos32[2 * i - (i & 63)] = p;
                    pos32[2 * i - (i & 63) + 64] = p;
                }
            } else if (i < n) {
                if constexpr (F32)
                    pos32[i] = make_float4((float)x[0][a], (float)x[1][a], (float)x[2][a], 0.0f);
                else
                    pos64[i] = make_double4(x[0][a], x[1][a], x[2][a], 0.0);
            }
        }
        sync();
        double e[1][A], o[1];
        if (ring) {
            if constexpr (kRing) pairs_ring<POT>(n, pos32, rbuf, e[0][0], g, rho);
        } else if (tiles) {
            if constexpr (kTiles) pairs_tiles<W, A>(n, pos32, rbuf, e[0], g);
        } else if constexpr (F32) {
            pairs_mixed<A, T, POT>(n, pos32, x, e[0], g, rho, li);
        } else {
            fp64_pairs<POT == kPairMorse>(x, e[0], g);
        }
#pragma unroll
        for (int a = 0; a < A; ++a)
            if (!active(a)) e[0][a] = g[0][a] = g[1][a] = g[2][a] = 0.0;
        sum_energy(e, o);
        if constexpr (!F32 && POT == kPairLJ) {
            // only a pair distance outside the range of recip_in_range can make
            // 1/r2 differ from the IEEE quotient, and it makes E not finite:
            // then the evaluation is repeated with the IEEE division
            if (!isfinite(o[0])) {
                fp64_pairs<true>(x, e[0], g);
#pragma unroll
                for (int a = 0; a < A; ++a)
                    if (!active(a)) e[0][a] = g[0][a] = g[1][a] = g[2][a] = 0.0;
                sum_energy(e, o);
            }
        }
        return (POT == kPairMorse ? 0.5 : 2.0) * o[0];
    }

    template <bool IEEE>
    __device__ __forceinline__ void fp64_pairs(const double (&x)[3][A], double (&e)[A],
                                               double (&g)[3][A]) {
        if constexpr (UP) {
            if (n <= up_n) {
                pairs_morse64_up(n, pos64, upm, uplist, x, e, g, rho, li);
                return;
            }
        }
        pairs_fp64<A, T, POT, IEEE>(n, pos64, x, e, g, rho, li);
    }

    __device__ __forceinline__ void sum_energy(double (&e)[1][A], double (&o)[1]) {
        if constexpr (G > 1)
            o[0] = group_sum<G>(e[0][0]);
        else
            team_sum<W, A, 1, NVMAX, L>(e, o, *sc, bank);
    }
};

// ---------------------------------------------------------------------------
// L-BFGS history.  rho is kept by age (slot 0 = newest) in registers; the
// vectors either by age in registers (HREG, shifted on every push) or in a
// global ring owned by the persistent workgroup.
// ---------------------------------------------------------------------------
template <int W, int A, bool HREG>
struct History;

template <int W, int A>
struct History<W, A, true> {
    double S[kMaxM][3][A];
    double Y[kMaxM][3][A];
    double rho[kMaxM];
    int hist = 0;
    double gamma = 1.0;

    __device__ __forceinline__ void init(double*, int) { hist = 0; gamma = 1.0; }
    __device__ __forceinline__ void clear() { hist = 0; }

    __device__ __forceinline__ void push(const double (&s)[3][A], const double (&y)[3][A], double r,
                                         double gam, int m) {
#pragma unroll
        for (int k = kMaxM - 1; k > 0; --k) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < A; ++a) {
                    S[k][c][a] = S[k - 1][c][a];
                    Y[k][c][a] = Y[k - 1][c][a];
                }
            rho[k] = rho[k - 1];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) {
                S[0][c][a] = s[c][a];
                Y[0][c][a] = y[c][a];
            }
        rho[0] = r;
        gamma = gam;
        hist = hist < m ? hist + 1 : m;
    }

    // r <- H r with all kMaxM pairs present: the same operations as apply(),
    // with no per-pair guards (no branches or register copies between pairs).
    template <class TM>
    __device__ __forceinline__ void apply_full(TM& tm, double (&r)[3][A]) {
        double al[kMaxM];
#pragma unroll
        for (int k = 0; k < kMaxM; ++k) {
            const double a = rho[k] * tm.dot(S[k], r);
            al[k] = a;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < A; ++q) r[c][q] = fma(-a, Y[k][c][q], r[c][q]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < A; ++q) r[c][q] = gamma * r[c][q];
#pragma unroll
        for (int k = kMaxM - 1; k >= 0; --k) {
            const double b = rho[k] * tm.dot(Y[k], r);
            const double w = al[k] - b;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < A; ++q) r[c][q] = fma(w, S[k][c][q], r[c][q]);
        }
    }

    // r <- H r (r holds g on entry).
    template <class TM>
    __device__ __forceinline__ void apply(TM& tm, double (&r)[3][A]) {
        const int h = tm.uni(hist);
        if (h == kMaxM) {
            apply_full(tm, r);
            return;
        }
        double al[kMaxM];
#pragma unroll
        for (int k = 0; k < kMaxM; ++k) {
            if (k < h) {
                const double a = rho[k] * tm.dot(S[k], r);
                al[k] = a;
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q = 0; q < A; ++q) r[c][q] = fma(-a, Y[k][c][q], r[c][q]);
            }
        }
        if (h > 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < A; ++q) r[c][q] = gamma * r[c][q];
        }
#pragma unroll
        for (int k = kMaxM - 1; k >= 0; --k) {
            if (k < h) {
                const double b = rho[k] * tm.dot(Y[k], r);
                const double w = al[k] - b;
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q = 0; q < A; ++q) r[c][q] = fma(w, S[k][c][q], r[c][q]);
            }
        }
    }
};

template <int W, int A>
struct History<W, A, false> {
    static constexpr int T = kWave * W;
    double* base;  // this workgroup's ring: S slots then Y slots, [slot][3][A][T]
    double rho[kMaxM];
    int hist = 0;
    int newest = -1;
    int m = 1;
    double gamma = 1.0;

    __device__ __forceinline__ double* vec(int slot, bool isY) const {
        return base + ((size_t)((isY ? kMaxM : 0) + slot) * 3 * A) * T + threadIdx.x;
    }
    __device__ __forceinline__ void init(double* b, int mm) {
        base = b;
        m = mm > 0 ? mm : 1;
        hist = 0;
        newest = -1;
        gamma = 1.0;
    }
    __device__ __forceinline__ void clear() { hist = 0; }

    __device__ __forceinline__ void push(const double (&s)[3][A], const double (&y)[3][A], double r,
                                         double gam, int mm) {
        newest = (newest + 1) % m;
        double* ps = vec(newest, false);
        double* py = vec(newest, true);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) {
                ps[(c * A + a) * T] = s[c][a];
                py[(c * A + a) * T] = y[c][a];
            }
#pragma unroll
        for (int k = kMaxM - 1; k > 0; --k) rho[k] = rho[k - 1];
        rho[0] = r;
        gamma = gam;
        hist = hist < mm ? hist + 1 : mm;
    }

    template <class TM>
    __device__ __forceinline__ void apply(TM& tm, double (&r)[3][A]) {
        const int h = tm.uni(hist);
        double al[kMaxM];
        double v[3][A];
#pragma unroll
        for (int k = 0; k < kMaxM; ++k) {
            if (k < h) {
                const int slot = (newest - k + m) % m;
                const double* ps = vec(slot, false);
                const double* py = vec(slot, true);
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q = 0; q < A; ++q) v[c][q] = ps[(c * A + q) * T];
                const double a = rho[k] * tm.dot(v, r);
                al[k] = a;
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q = 0; q < A; ++q) r[c][q] = fma(-a, py[(c * A + q) * T], r[c][q]);
            }
        }
        if (h > 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < A; ++q) r[c][q] = gamma * r[c][q];
        }
#pragma unroll
        for (int k = kMaxM - 1; k >= 0; --k) {
            if (k < h) {
                const int slot = (newest - k + m) % m;
                const double* ps = vec(slot, false);
                const double* py = vec(slot, true);
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q = 0; q < A; ++q) v[c][q] = py[(c * A + q) * T];
                const double b = rho[k] * tm.dot(v, r);
                const double w = al[k] - b;
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q = 0; q < A; ++q) r[c][q] = fma(w, ps[(c * A + q) * T], r[c][q]);
            }
        }
    }
};

// Phase outcomes (LJ_* statuses, plus the FP32 phase's stall exit).
constexpr int kStall = 100;
// Relative energy change that the FP64 line search treats as rounding noise.
constexpr double kLsResolution = 0x1.0p-50;
// The FP32 phase treats energy changes as noise-limited only once
// ||g|| < kNoiseZone * its tolerance: there the Armijo allowance and the exit
// after five accepted steps without a decrease apply.
constexpr double kNoiseZone = 100.0;
// Inside the noise zone the FP32 phase also ends after kZonePatience accepted
// steps without lowering the best gradient norm of the zone by 10 %.
constexpr int kZonePatience = 30;

// E and g at x with FP32 pair arithmetic when f32 (only compiled when CAN32).
template <bool CAN32, int W, int A, int POT, int L, int G, bool UP>
__device__ __forceinline__ double eval_phase(Team<W, A, POT, L, G, UP>& tm, const double (&x)[3][A],
                                             double (&g)[3][A], bool f32) {
    if constexpr (CAN32) {
        if (f32) return tm.template eval<true>(x, g);
    }
    return tm.template eval<false>(x, g);
}

// One L-BFGS run from x (history cleared).  On return x, g, E hold the last
// accepted iterate.  f32 (a uniform runtime flag, so the mixed kernel holds a
// single copy of this loop for both phases) selects the FP32 pair arithmetic,
// the Armijo noise allowance and the stall exit of the mixed path's first
// phase.
template <bool CAN32, int W, int A, bool HREG, int POT, int L, int G, bool UP>
__device__ int lbfgs_run(Team<W, A, POT, L, G, UP>& tm, History<W, A, HREG>& H, double (&x)[3][A],
                         double (&g)[3][A], double& E, double& gnorm, int& iters, int& evals,
                         const LbfgsDev& p, double gtol, int max_iter, bool f32_flag) {
    const bool F32 = CAN32 && f32_flag;
    double d[3][A], xt[3][A], gt[3][A];
    H.clear();
    E = eval_phase<CAN32>(tm, x, g, F32);
    ++evals;
    double gg = tm.dot(g, g);  // later iterations get it from the curvature reduction
    gnorm = sqrt(gg);
    int it = 0;
    int stall = 0;
    int zone_wait = 0;
    double zone_best = 1.0e300;
    const double ms2 = p.max_step * p.max_step;
    for (;;) {
        if (!isfinite(E) || !isfinite(gg)) {
            iters += it;
            return LJ_NONFINITE;
        }
        if (gnorm < gtol) {
            iters += it;
            return LJ_CONVERGED;
        }
        if (it >= max_iter) {
            iters += it;
            return LJ_MAXITER;
        }
        // d = -H g
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) d[c][a] = g[c][a];
        H.apply(tm, d);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) d[c][a] = -d[c][a];
        double gd, dmax2;
        tm.dot_max(g, d, gd, dmax2, ms2);
        if (tm.uni(H.hist) > 0 && !(gd < 0.0)) {
            H.clear();
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < A; ++a) d[c][a] = -g[c][a];
            tm.dot_max(g, d, gd, dmax2, ms2);
        }
        if (dmax2 > ms2) {
            const double sc = p.max_step / sqrt(dmax2);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < A; ++a) d[c][a] = d[c][a] * sc;
            gd = tm.dot(g, d);
        }
        // backtracking Armijo line search
        const bool noise_zone = F32 && gnorm < kNoiseZone * gtol;
        double alpha = 1.0, Et = 0.0;
        bool ok = false;
        // relative energy change below which the energy comparison is decided
        // by rounding: 4 ulps of E in FP64, the FP32 noise allowance in the
        // FP32 phase
        const double resolution = F32 ? p.ls_noise : kLsResolution;
        for (int ls = 0; ls < p.max_ls; ++ls) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < A; ++a) xt[c][a] = fma(alpha, d[c][a], x[c][a]);
            Et = eval_phase<CAN32>(tm, xt, gt, F32);
            ++evals;
            double rhs = fma(p.c1 * alpha, gd, E);
            // FP32 phase near its tolerance: the full quasi-Newton step may be
            // accepted within the FP32 energy noise; a backtracked step, or any
            // step farther from convergence, must show a real decrease
            if (noise_zone && alpha == 1.0) rhs = rhs + p.ls_noise * fabs(E);
            if (Et <= rhs) {
                ok = true;
                break;
            }
            // An energy change within the resolution of E cannot decide the
            // test; the gradients can (approximate Armijo condition:
            // g_t.d <= (2 c1 - 1) g.d).  In the FP32 phase this carries the
            // descent on below the gradient norm at which energy changes
            // vanish in the FP32 noise (about 0.04 at LJ38), down to the
            // phase's tolerance, so the FP64 polish starts close to the minimum
            if (fabs(Et - E) <= resolution * fabs(E) &&
                tm.dot(gt, d) <= (2.0 * p.c1 - 1.0) * gd) {
                ok = true;
                break;
            }
            alpha = alpha * 0.5;
        }
        // FP32 phase while atoms still overlap (E > 0): a step that lowers E
        // by less than the FP32 resolution of E made no measurable progress
        // (its direction was scaled down by the curvature of one extremely
        // stiff pair) and counts as a failed line search, so the history is
        // dropped for a steepest-descent restart
        if (ok && F32 && E > 0.0 && !(E - Et > p.ls_noise * E)) ok = false;
        if (!ok) {
            if (tm.uni(H.hist) > 0) {
                H.clear();
                continue;
            }
            iters += it;
            return LJ_LSFAIL;
        }
        // s = xt - x (into d), y = gt - g (into g)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) {
                d[c][a] = xt[c][a] - x[c][a];
                g[c][a] = gt[c][a] - g[c][a];
            }
        double sy, yy, ss, ggt;
        tm.dot4(d, g, gt, sy, yy, ss, ggt);
        if (ss == 0.0) {
            // Null step: the accepted trial point equals x, so no progress is
            // possible along d; treated as a failed line search.  g holds y
            // here; x_t == x implies g_t == g, so restore g from g_t.
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < A; ++a) g[c][a] = gt[c][a];
            if (tm.uni(H.hist) > 0) {
                H.clear();
                continue;
            }
            iters += it;
            return LJ_LSFAIL;
        }
        // the square roots and quotients of this step are independent of one
        // another: formed together so their latencies overlap
        const double gn_t = sqrt(ggt);
        const double syy = sqrt(ss * yy);
        const double rho_t = 1.0 / sy;
        const double gam_t = sy / yy;
        if (p.m > 0 && sy > p.curv_eps * syy) H.push(d, g, rho_t, gam_t, p.m);
        stall = (Et < E || !noise_zone) ? 0 : stall + 1;
        if (noise_zone) {
            if (gnorm < 0.9 * zone_best) {
                zone_best = gnorm;
                zone_wait = 0;
            } else {
                ++zone_wait;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) {
                x[c][a] = xt[c][a];
                g[c][a] = gt[c][a];
            }
        E = Et;
        gg = ggt;
        gnorm = gn_t;
        ++it;
        if (stall >= 5 || zone_wait >= kZonePatience) {  // FP32 phase's noise zone only
            iters += it;
            return kStall;
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent minimiser kernel: one launch per size class.  A workgroup claims
// the next cluster of its class from the queue (G > 1: the next G clusters,
// one per packed team of 64 / G lanes) and minimises it; it claims again once
// all of its teams are done.
// ---------------------------------------------------------------------------
template <int MIXED, int W, int A, bool HREG, int POT, int L = kWave, int G = 1, int OCC = 1>
__global__ __launch_bounds__(kWave* W) __attribute__((amdgpu_waves_per_eu(OCC))) void minimize_kernel(
    MinArgs args) {
    constexpr int T = kWave * W;
    constexpr int LG = kWave / G;  // lanes of a packed team
    __shared__ double4 pos_buf[T * A];
    __shared__ TeamScratch<W, 4 * A> scratch;
    __shared__ int claim;
    __shared__ float tile_rbuf[(MIXED && G == 1 &&
                                ((POT == kPairLJ && kUseTiles<W, A>) || (W == 1 && A == 1)))
                                   ? 6 * T * A
                                   : 1];

    // one-wavefront, one-cluster Morse kernels at one wavefront per SIMD take
    // the unique-pair FP64 evaluation, with its matrix in dynamic LDS (for
    // Eq. (1) the ordered loop is as fast: its pair terms are too cheap to
    // pay for the matrix's LDS traffic)
    constexpr bool kUp = W == 1 && A == 1 && G == 1 && OCC == 1 && POT == kPairMorse;
    extern __shared__ double2 up_matrix[];
    const int team = G > 1 ? (int)threadIdx.x / LG : 0;
    Team<W, A, POT, L, G, kUp> tm;
    tm.upm = up_matrix;
    tm.up_n = kUp ? args.up_n : 0;
    tm.uplist = reinterpret_cast<uint2*>(up_matrix + (size_t)tm.up_n * tm.up_n);
    tm.li = G > 1 ? (int)threadIdx.x % LG : (int)threadIdx.x;
    tm.pos64 = pos_buf + team * LG;
    tm.pos32 = reinterpret_cast<float4*>(pos_buf) + team * LG;
    tm.rbuf = tile_rbuf;
    tm.sc = &scratch;
    tm.bank = 0;
    tm.rho = args.rho;
    History<W, A, HREG> H;
    constexpr size_t kHistPerWG = (size_t)2 * kMaxM * 3 * A * T;
    H.init(args.hist ? args.hist + kHistPerWG * blockIdx.x : nullptr, args.p.m);

    const int start = args.plan.cls[args.cls];
    const int count = args.plan.cls[kNumClasses + args.cls];
    const int64_t total = args.total;
    for (;;) {
        if (threadIdx.x == 0) claim = atomicAdd(&args.plan.queue[args.cls], G);
        __syncthreads();
        const int idx0 = claim;
        __syncthreads();
        if (idx0 >= count) break;
        const int idx = idx0 + team;
        const bool has = idx < count;  // a packed team past the end idles
        const int b = has ? args.plan.list[start + idx] : 0;
        const int o = has ? args.offset[b] : 0;
        const int n = has ? args.offset[b + 1] - o : 0;
        tm.n = n;  // the plan guarantees 0 <= n <= T*A (G > 1: <= 64 / G)
        tm.prepare();

        double x[3][A], g[3][A];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) {
                const int i = a * T + tm.li;
                x[c][a] = i < n ? args.xyz[c * total + o + i] : 0.0;
                if (args.u.scaled) x[c][a] = x[c][a] / args.u.sigma;
            }
        double E = 0.0, gn = 0.0;
        int iters = 0, evals = 0, st = LJ_CONVERGED;
        // Mixed: phase 0 is the FP32 phase, phase 1 the FP64 polish from its
        // end point (one call site, so one copy of the L-BFGS loop).
        for (int phase = MIXED ? 0 : 1; phase < 2; ++phase) {
            const bool f32 = phase == 0;
            const double gt = f32 ? fmax(args.p.gtol, args.p.gtol_mixed_per_atom * (double)n)
                                  : args.p.gtol;
            const int r = lbfgs_run<MIXED != 0>(tm, H, x, g, E, gn, iters, evals, args.p, gt,
                                                args.p.max_iter, f32);
            if (!f32) {
                st = r;
                break;
            }
            if (args.xyz_switch) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int a = 0; a < A; ++a) {
                        const int i = a * T + tm.li;
                        if (i < n)
                            args.xyz_switch[c * total + o + i] =
                                args.u.scaled ? x[c][a] * args.u.sigma : x[c][a];
                    }
            }
            if (!args.p.polish) {
                // report the FP32 end point re-evaluated in FP64
                E = tm.template eval<false>(x, g);
                ++evals;
                const double gg = tm.dot(g, g);
                gn = sqrt(gg);
                if (!isfinite(E) || !isfinite(gg))
                    st = LJ_NONFINITE;
                else if (gn < args.p.gtol)
                    st = LJ_CONVERGED;
                else if (r == LJ_CONVERGED || r == kStall || r == LJ_LSFAIL)
                    st = LJ_SWITCHED;  // the FP32 phase reached its tolerance or resolution
                else
                    st = r == LJ_NONFINITE ? LJ_LSFAIL : r;
                break;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) {
                const int i = a * T + tm.li;
                if (i < n)
                    args.xyz[c * total + o + i] = args.u.scaled ? x[c][a] * args.u.sigma : x[c][a];
            }
        if (has && tm.li == 0) {
            args.energy[b] = E * args.u.escale;
            args.gnorm[b] = gn * args.u.gscale;
            args.iters[b] = iters;
            args.evals[b] = evals;
            args.status[b] = st;
        }
    }
}

// ---------------------------------------------------------------------------
// Plan: list the (active) clusters by N descending and split the list into
// size classes.  One workgroup; rejects clusters whose N is outside
// [0, max_n] with a per-cluster status instead of running them.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void plan_kernel(const int32_t* offset, int num, int max_n,
                                                    const int32_t* active, Plan plan,
                                                    int32_t* status) {
    __shared__ int cnt[LJ_MAX_ATOMS_MIN + 1];
    const int t = threadIdx.x;
    for (int k = t; k <= LJ_MAX_ATOMS_MIN; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    for (int b = t; b < num; b += blockDim.x) {
        if (active && !active[b]) continue;
        const int n = offset[b + 1] - offset[b];
        if (n < 0 || n > max_n) {
            if (status) status[b] = kStatusBadSize;
            continue;
        }
        atomicAdd(&cnt[n], 1);
    }
    __syncthreads();
    if (t == 0) {
        // descending exclusive scan of the size counts; sizes above max_n were
        // rejected, so their counts (and scan values) are zero: start at max_n
        const int top = max_n < LJ_MAX_ATOMS_MIN ? max_n : LJ_MAX_ATOMS_MIN;
        int run = 0;
        for (int k = top; k >= 0; --k) {
            const int c = cnt[k];
            cnt[k] = run;
            run += c;
        }
        // classes: (256, 1024], (128, 256], (64, 128], [0, 64]
        const int s3 = 0, s2 = cnt[256], s1 = cnt[128], s0 = cnt[64];
        plan.cls[3] = s3;
        plan.cls[2] = s2;
        plan.cls[1] = s1;
        plan.cls[0] = s0;
        plan.cls[kNumClasses + 3] = s2 - s3;
        plan.cls[kNumClasses + 2] = s1 - s2;
        plan.cls[kNumClasses + 1] = s0 - s1;
        plan.cls[kNumClasses + 0] = run - s0;
        for (int c = 0; c < kNumClasses; ++c) plan.queue[c] = 0;
    }
    __syncthreads();
    for (int b = t; b < num; b += blockDim.x) {
        if (active && !active[b]) continue;
        const int n = offset[b + 1] - offset[b];
        if (n < 0 || n > max_n) continue;
        const int pos = atomicAdd(&cnt[n], 1);
        plan.list[pos] = b;
    }
}

// ---------------------------------------------------------------------------
// Batched energy + gradient: one workgroup per cluster.
// ---------------------------------------------------------------------------
template <int MIXED, int W, int A, int POT>
__global__ __launch_bounds__(kWave* W) void energy_grad_kernel(const int32_t* offset, int64_t total,
                                                               const double* xyz, double* energy,
                                                               double* grad, double rho, Units u) {
    constexpr int T = kWave * W;
    __shared__ double4 pos_buf[T * A];
    __shared__ TeamScratch<W, 4 * A> scratch;
    __shared__ float tile_rbuf[(MIXED && ((POT == kPairLJ && kUseTiles<W, A>) || (W == 1 && A == 1)))
                                   ? 6 * T * A
                                   : 1];
    const int b = blockIdx.x;
    const int o = offset[b];
    const int n = offset[b + 1] - o;
    if (n < 0 || n > T * A) {  // offsets disagree with the host max_n
        if (threadIdx.x == 0) energy[b] = __builtin_nan("");
        return;
    }
    Team<W, A, POT> tm;
    tm.upm = nullptr;
    tm.uplist = nullptr;
    tm.up_n = 0;
    tm.pos64 = pos_buf;
    tm.pos32 = reinterpret_cast<float4*>(pos_buf);
    tm.rbuf = tile_rbuf;
    tm.sc = &scratch;
    tm.bank = 0;
    tm.n = n;
    tm.li = threadIdx.x;
    tm.rho = rho;
    double x[3][A], g[3][A];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const int i = a * T + threadIdx.x;
            x[c][a] = i < n ? xyz[c * total + o + i] : 0.0;
            if (u.scaled) x[c][a] = x[c][a] / u.sigma;
        }
    const double E = tm.template eval<MIXED != 0>(x, g);
    if (threadIdx.x == 0) energy[b] = E * u.escale;
    if (grad) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) {
                const int i = a * T + threadIdx.x;
                if (i < n) grad[c * total + o + i] = g[c][a] * u.gscale;
            }
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (internal C++ interface used by the C ABI layer).
// ---------------------------------------------------------------------------
EvalShape eval_shape(int max_n) {
    const int n = max_n < 1 ? 1 : max_n;
    if (n <= 64) return {1, 1};
    if (n <= 128) return {2, 1};
    if (n <= 256) return {4, 1};
    if (n <= 512) return {8, 1};
    if (n <= 1024) return {16, 1};
    if (n <= 2048) return {16, 2};
    return {16, 4};
}

bool eval_shape_supported(EvalShape s) {
    const bool w = s.W == 1 || s.W == 2 || s.W == 4 || s.W == 8 || s.W == 16;
    const bool a = s.A == 1 || s.A == 2 || s.A == 4;
    return w && a;
}

template <int MIXED, int POT>
static hipError_t launch_eval_t(EvalShape s, int num, const int32_t* off, int64_t total,
                                const double* xyz, double* e, double* g, double rho, Units u,
                                hipStream_t st) {
    dim3 grid(num), block(kWave * s.W);
#define LJ_EVAL_CASE(WW, AA)                                                                  \
    if (s.W == WW && s.A == AA) {                                                             \
        hipLaunchKernelGGL((energy_grad_kernel<MIXED, WW, AA, POT>), grid, block, 0, st, off, \
                           total, xyz, e, g, rho, u);                                         \
        return hipGetLastError();                                                             \
    }
    LJ_EVAL_CASE(1, 1)
    LJ_EVAL_CASE(2, 1)
    LJ_EVAL_CASE(4, 1)
    LJ_EVAL_CASE(8, 1)
    LJ_EVAL_CASE(16, 1)
    LJ_EVAL_CASE(1, 2)
    LJ_EVAL_CASE(2, 2)
    LJ_EVAL_CASE(4, 2)
    LJ_EVAL_CASE(8, 2)
    LJ_EVAL_CASE(16, 2)
    LJ_EVAL_CASE(1, 4)
    LJ_EVAL_CASE(2, 4)
    LJ_EVAL_CASE(4, 4)
    LJ_EVAL_CASE(8, 4)
    LJ_EVAL_CASE(16, 4)
#undef LJ_EVAL_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_energy_grad(int mixed, int pot, EvalShape s, int num, const int32_t* off,
                              int64_t total, const double* xyz, double* e, double* g, double rho,
                              Units u, hipStream_t st) {
    if (pot == kPairMorse)
        return mixed ? launch_eval_t<1, kPairMorse>(s, num, off, total, xyz, e, g, rho, u, st)
                     : launch_eval_t<0, kPairMorse>(s, num, off, total, xyz, e, g, rho, u, st);
    return mixed ? launch_eval_t<1, kPairLJ>(s, num, off, total, xyz, e, g, rho, u, st)
                 : launch_eval_t<0, kPairLJ>(s, num, off, total, xyz, e, g, rho, u, st);
}

// Minimiser shapes.  Classes 0-2 keep the history in registers; class 3
// (N in 257..1024) keeps it in a global ring.  Each class has interchangeable
// shapes (the schedule table or the built-in rule picks one per call):
//   class 0 (N <= 64):   0  one wavefront per cluster
//                        1  one wavefront, reductions over one 16-lane row
//                           (N <= 16)
//                        2  two clusters per wavefront, 32 lanes each (N <= 32)
//                        3  four clusters per wavefront, 16 lanes each (N <= 16)
//                        4-7  shapes 0-3 compiled for two wavefronts per SIMD
//                           (at most 256 registers, the rest spilled): for
//                           batches of more wavefronts than SIMDs
//   class 1 (N <= 128):  0  two wavefronts;  1  one wavefront, two atoms per lane
//   class 2 (N <= 256):  0  four wavefronts;  1  three wavefronts (N <= 192)
//   class 3 (N <= 1024): 0  16 wavefronts x 1 atom, 1  8 x 2, 2  4 x 4
struct ClassShape {
    int W, A;
    bool hreg;
    int G;     // clusters per workgroup
    int max_n; // largest cluster the shape holds
};
constexpr int kMaxShapes = 8;
constexpr int kShapes[kNumClasses] = {8, 2, 2, 3};
constexpr ClassShape kShape[kNumClasses][kMaxShapes] = {
    {{1, 1, true, 1, 64}, {1, 1, true, 1, 16}, {1, 1, true, 2, 32}, {1, 1, true, 4, 16},
     {1, 1, true, 1, 64}, {1, 1, true, 1, 16}, {1, 1, true, 2, 32}, {1, 1, true, 4, 16}},
    {{2, 1, true, 1, 128}, {1, 2, true, 1, 128}},
    {{4, 1, true, 1, 256}, {3, 1, true, 1, 192}},
    {{16, 1, false, 1, 1024}, {8, 2, false, 1, 1024}, {4, 4, false, 1, 1024}}};

int class_shapes(int c) { return c >= 0 && c < kNumClasses ? kShapes[c] : 0; }
int shape_max_n(int c, int shape) { return kShape[c][shape].max_n; }
int shape_clusters_per_wg(int c, int shape) { return kShape[c][shape].G; }

int class_of(int n) {
    for (int c = 0; c < kNumClasses; ++c)
        if (n <= kClassMaxN[c]) return c;
    return -1;
}

size_t class_hist_bytes_per_wg(int c, int shape) {
    const ClassShape s = kShape[c][shape];
    return s.hreg ? 0 : (size_t)2 * kMaxM * 3 * s.A * kWave * s.W * sizeof(double);
}

template <int MIXED, int W, int A, bool HREG, int POT, int L = kWave, int G = 1, int OCC = 1>
static const void* min_kernel_ptr() {
    return reinterpret_cast<const void*>(&minimize_kernel<MIXED, W, A, HREG, POT, L, G, OCC>);
}

template <int MIXED, int POT>
static const void* minimize_kernel_pm(int c, int shape) {
    switch (c * kMaxShapes + shape) {
        case 0: return min_kernel_ptr<MIXED, 1, 1, true, POT>();
        case 1: return min_kernel_ptr<MIXED, 1, 1, true, POT, 16>();
        case 2: return min_kernel_ptr<MIXED, 1, 1, true, POT, kWave, 2>();
        case 3: return min_kernel_ptr<MIXED, 1, 1, true, POT, kWave, 4>();
        case 4: return min_kernel_ptr<MIXED, 1, 1, true, POT, kWave, 1, 2>();
        case 5: return min_kernel_ptr<MIXED, 1, 1, true, POT, 16, 1, 2>();
        case 6: return min_kernel_ptr<MIXED, 1, 1, true, POT, kWave, 2, 2>();
        case 7: return min_kernel_ptr<MIXED, 1, 1, true, POT, kWave, 4, 2>();
        case kMaxShapes + 0: return min_kernel_ptr<MIXED, 2, 1, true, POT>();
        case kMaxShapes + 1: return min_kernel_ptr<MIXED, 1, 2, true, POT>();
        case 2 * kMaxShapes + 0: return min_kernel_ptr<MIXED, 4, 1, true, POT>();
        case 2 * kMaxShapes + 1: return min_kernel_ptr<MIXED, 3, 1, true, POT>();
        case 3 * kMaxShapes + 0: return min_kernel_ptr<MIXED, 16, 1, false, POT>();
        case 3 * kMaxShapes + 1: return min_kernel_ptr<MIXED, 8, 2, false, POT>();
        case 3 * kMaxShapes + 2: return min_kernel_ptr<MIXED, 4, 4, false, POT>();
    }
    return nullptr;
}

const void* minimize_kernel_for(int mixed, int pot, int c, int shape) {
    if (c < 0 || c >= kNumClasses || shape < 0 || shape >= kShapes[c]) return nullptr;
    if (pot == kPairMorse)
        return mixed ? minimize_kernel_pm<1, kPairMorse>(c, shape)
                     : minimize_kernel_pm<0, kPairMorse>(c, shape);
    return mixed ? minimize_kernel_pm<1, kPairLJ>(c, shape) : minimize_kernel_pm<0, kPairLJ>(c, shape);
}

int class_block(int c, int shape) { return kWave * kShape[c][shape].W; }

int class_up_n(int c, int shape, int max_n, int pot) {
    if (pot != kPairMorse || c < 0 || c >= kNumClasses || shape < 0 || shape >= kShapes[c])
        return 0;
    const ClassShape s = kShape[c][shape];
    // the one-wavefront, one-cluster shapes at one wavefront per SIMD
    if (!(s.W == 1 && s.A == 1 && s.G == 1 && !(c == 0 && shape >= 4))) return 0;
    int n = max_n < s.max_n ? max_n : s.max_n;
    if (n > kUpMaxN) n = kUpMaxN;
    return n >= 2 ? n : 0;
}

size_t class_dyn_lds(int c, int shape, int max_n, int pot) {
    const size_t n = (size_t)class_up_n(c, shape, max_n, pot);
    return n * n * sizeof(double2) + n * (n > 0 ? n - 1 : 0) / 2 * sizeof(uint2);
}

hipError_t launch_plan(const int32_t* offset, int num, int max_n, const int32_t* active, Plan plan,
                       int32_t* status, hipStream_t st) {
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, st, offset, num, max_n, active, plan,
                       status);
    return hipGetLastError();
}

hipError_t launch_minimize_class(int mixed, int c, int shape, int grid, const MinArgs& a,
                                 hipStream_t st) {
    const void* k = minimize_kernel_for(mixed, a.pot, c, shape);
    if (!k) return hipErrorInvalidValue;
    MinArgs b = a;
    b.up_n = class_up_n(c, shape, a.max_n, a.pot);
    void* args[] = {&b};
    return hipLaunchKernel(k, dim3(grid), dim3(class_block(c, shape)), args,
                           class_dyn_lds(c, shape, a.max_n, a.pot), st);
}

}  // namespace lj
