// Device building blocks for gfx950: team reductions in a fixed tree order,
// the LDS-staged pair loops (Eq. (1) and the Morse pair, FP64 and FP32),
// Philox4x64-10 and the deterministic exp of the Metropolis test and the
// Morse pair.
//
// A "team" is the W wavefronts (64 lanes each) of one workgroup that work on
// one cluster.  Atom i of a cluster lives in thread t = i mod T, slot
// a = i / T (T = 64 W); each thread keeps its A slots in registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lj_bh.h"

namespace lj {

constexpr int kWave = 64;
constexpr int kMaxM = 10;   // L-BFGS history held per cluster (LJ_MAX_M)
constexpr int kTileJ = 64;  // FP32 partner tile before a per-atom FP64 flush

// ---------------------------------------------------------------------------
// Lane 0's value as a wavefront-uniform (scalar) value: a value that every
// lane already holds, or a 16-leaf sum that row 0 holds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double uniform(double v) {
    int2 b = *reinterpret_cast<int2*>(&v);
    b.x = __builtin_amdgcn_readfirstlane(b.x);
    b.y = __builtin_amdgcn_readfirstlane(b.y);
    return *reinterpret_cast<double*>(&b);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Sum over the 64 lanes in balanced-tree order, entirely in registers.
// Levels 1-4 run inside each 16-lane row with DPP lane permutes:
// quad_perm [1,0,3,2] and [2,3,0,1] pair lanes 2^0 and 2^1 apart; once every
// quad holds one value, row_half_mirror pairs each quad with the other quad
// of its 8-lane half, and once every half holds one value, row_mirror pairs
// the two halves of the row.  Levels 5-6 use the gfx950 permlane swaps:
// v_permlane16_swap exchanges odd rows of one copy with even rows of another,
// so the sum of the two results pairs rows (0,1) and (2,3); v_permlane32_swap
// does the same for the two 32-lane halves.  Each level adds two values that
// are both held by the lanes involved (IEEE addition is commutative), so
// every lane ends with identical bits: the pairwise sum over the lane index.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    int2 b = *reinterpret_cast<int2*>(&v);
    b.x = __builtin_amdgcn_mov_dpp(b.x, CTRL, 0xF, 0xF, true);
    b.y = __builtin_amdgcn_mov_dpp(b.y, CTRL, 0xF, 0xF, true);
    return *reinterpret_cast<double*>(&b);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppMirror = 0x140;     // row_mirror

// (value of the partner row, own value) ordered so that adding them gives the
// same bits in both rows of a pair: returns the two swapped copies.
__device__ __forceinline__ void swap_rows16(double v, double& lo, double& hi) {
    int2 b = *reinterpret_cast<int2*>(&v);
    auto x = __builtin_amdgcn_permlane16_swap(b.x, b.x, false, false);
    auto y = __builtin_amdgcn_permlane16_swap(b.y, b.y, false, false);
    int2 l = make_int2((int)x[0], (int)y[0]);
    int2 h = make_int2((int)x[1], (int)y[1]);
    lo = *reinterpret_cast<double*>(&l);
    hi = *reinterpret_cast<double*>(&h);
}

__device__ __forceinline__ void swap_halves32(double v, double& lo, double& hi) {
    int2 b = *reinterpret_cast<int2*>(&v);
    auto x = __builtin_amdgcn_permlane32_swap(b.x, b.x, false, false);
    auto y = __builtin_amdgcn_permlane32_swap(b.y, b.y, false, false);
    int2 l = make_int2((int)x[0], (int)y[0]);
    int2 h = make_int2((int)x[1], (int)y[1]);
    lo = *reinterpret_cast<double*>(&l);
    hi = *reinterpret_cast<double*>(&h);
}

// L = 64 leaves, or L = 16 when only lanes 0-15 can hold nonzero values (a
// cluster of at most 16 atoms): then the sum is the tree of row 0 (the same
// 16-leaf tree the pairwise sum pads N <= 16 to), read from lane 0 as a
// wavefront-uniform (scalar) value; branches on it are then scalar too.
template <int L = kWave>
__device__ __forceinline__ double wave_sum(double v) {
    static_assert(L == 16 || L == kWave, "16 or 64 leaves");
    v = v + dpp<kDppXor1>(v);
    v = v + dpp<kDppXor2>(v);
    v = v + dpp<kDppHalfMirror>(v);
    v = v + dpp<kDppMirror>(v);
    if constexpr (L == 16) return uniform(v);
    double a, b;
    swap_rows16(v, a, b);  // a: even row's value in both rows, b: odd row's
    v = a + b;
    swap_halves32(v, a, b);
    return a + b;
}

// G clusters packed in one wavefront (G = 2: lanes 32k .. 32k + 31; G = 4:
// one 16-lane row each): the sum over each cluster's lanes, in the pairwise
// order over its lane index.  The four row levels of wave_sum give each row's
// 16-leaf tree; for G = 2 the permlane16 swap then pairs rows 0 with 1 and 2
// with 3.  Every lane ends with its own cluster's sum.  These are the trees
// the pairwise sum pads N <= 16 (G = 4) or N <= 32 (G = 2) to.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G == 2 || G == 4, "2 or 4 clusters per wavefront");
    v = v + dpp<kDppXor1>(v);
    v = v + dpp<kDppXor2>(v);
    v = v + dpp<kDppHalfMirror>(v);
    v = v + dpp<kDppMirror>(v);
    if constexpr (G == 2) {
        double a, b;
        swap_rows16(v, a, b);
        v = a + b;
    }
    return v;
}

template <int G>
__device__ __forceinline__ double group_max(double v) {
    static_assert(G == 2 || G == 4, "2 or 4 clusters per wavefront");
    v = fmax(v, dpp<kDppXor1>(v));
    v = fmax(v, dpp<kDppXor2>(v));
    v = fmax(v, dpp<kDppHalfMirror>(v));
    v = fmax(v, dpp<kDppMirror>(v));
    if constexpr (G == 2) {
        double a, b;
        swap_rows16(v, a, b);
        v = fmax(a, b);
    }
    return v;
}

constexpr int kDppRor4 = 0x124;   // row_ror:4  (lane i of a row takes lane i - 4)
constexpr int kDppRor8 = 0x128;   // row_ror:8  (i takes i ^ 8)
constexpr int kDppRor12 = 0x12C;  // row_ror:12 (i takes i + 4)

// Lane l takes lane l ^ 4: the rotation by 12 fills banks 0 and 2 of every
// row (lanes 0-3, 8-11), the rotation by 4 then fills banks 1 and 3.
__device__ __forceinline__ double dpp_xor4(double v) {
    int2 b = *reinterpret_cast<int2*>(&v);
    int2 r;
    r.x = __builtin_amdgcn_mov_dpp(b.x, kDppRor12, 0xF, 0x5, false);
    r.y = __builtin_amdgcn_mov_dpp(b.y, kDppRor12, 0xF, 0x5, false);
    r.x = __builtin_amdgcn_update_dpp(r.x, b.x, kDppRor4, 0xF, 0xA, false);
    r.y = __builtin_amdgcn_update_dpp(r.y, b.y, kDppRor4, 0xF, 0xA, false);
    return *reinterpret_cast<double*>(&r);
}

constexpr int kDppNewBcast = 0x150;  // row_newbcast:k = 0x150 + k (lane k of each row to the row)

// Four sums over the 64 lanes, each with exactly the pairings of wave_sum,
// sharing one exchange per level: at the first level (lanes 2^0 apart) even
// lanes keep a and c and hand b and d to their odd partner, which keeps b and
// d; at the second (2^1 apart) each lane keeps one of its two partial sums and
// hands over the other, so that lane l then carries value l mod 4.  The
// remaining levels pair lanes 4, 8, 16 and 32 apart, which preserves the lane
// residue mod 4.  Each addition combines the same two blocks of lanes as in
// wave_sum (IEEE addition is commutative), so every result has wave_sum's
// bits.  Every row then holds the four totals in its lanes 0 .. 3, and
// row_newbcast hands each total to all lanes (a vector value, like
// wave_sum's: a scalar read-out changes how the compiler allocates the
// minimiser's registers and spills the L-BFGS state).
__device__ __forceinline__ void wave_sum4(double a, double b, double c, double d,
                                          double (&out)[4]) {
    const int lane = __lane_id();
    const bool odd = (lane & 1) != 0, hi = (lane & 2) != 0;
    const double u = (odd ? b : a) + dpp<kDppXor1>(odd ? a : b);
    const double w = (odd ? d : c) + dpp<kDppXor1>(odd ? c : d);
    double v = (hi ? w : u) + dpp<kDppXor2>(hi ? u : w);
    v = v + dpp_xor4(v);
    v = v + dpp<kDppRor8>(v);
    double x, y;
    swap_rows16(v, x, y);
    v = x + y;
    swap_halves32(v, x, y);
    v = x + y;
    out[0] = dpp<kDppNewBcast + 0>(v);
    out[1] = dpp<kDppNewBcast + 1>(v);
    out[2] = dpp<kDppNewBcast + 2>(v);
    out[3] = dpp<kDppNewBcast + 3>(v);
}

template <int L = kWave>
__device__ __forceinline__ double wave_max(double v) {
    static_assert(L == 16 || L == kWave, "16 or 64 leaves");
    v = fmax(v, dpp<kDppXor1>(v));
    v = fmax(v, dpp<kDppXor2>(v));
    v = fmax(v, dpp<kDppHalfMirror>(v));
    v = fmax(v, dpp<kDppMirror>(v));
    if constexpr (L == 16) return uniform(v);
    double a, b;
    swap_rows16(v, a, b);
    v = fmax(a, b);
    swap_halves32(v, a, b);
    return fmax(a, b);
}

// Balanced tree over K values (K a power of two): ((r0+r1)+(r2+r3))+...
template <int K>
__device__ __forceinline__ double tree(const double* r) {
    if constexpr (K == 1) {
        return r[0];
    } else {
        return tree<K / 2>(r) + tree<K / 2>(r + K / 2);
    }
}

// Balanced tree over the W wavefront sums of a team, padded with zeros to a
// power of two (a team of 3 wavefronts adds its third sum to a zero, as the
// pairwise sum over the atom index padded to 256 does).
template <int W>
__device__ __forceinline__ double tree_w(const double* r) {
    if constexpr ((W & (W - 1)) == 0) {
        return tree<W>(r);
    } else {
        constexpr int P = W < 2 ? 1 : W < 4 ? 4 : W < 8 ? 8 : 16;
        static_assert(W < P && P <= 16, "teams of at most 16 wavefronts");
        double q[P];
#pragma unroll
        for (int k = 0; k < P; ++k) q[k] = k < W ? r[k] : 0.0;
        return tree<P>(q);
    }
}

// Team reduction scratch in LDS: two alternating banks of NV x W doubles.
// One barrier per reduction: a bank is rewritten only two reductions later,
// and every thread has passed the intermediate reduction's barrier (after
// reading this bank) before that happens.
template <int W, int NVMAX>
struct TeamScratch {
    double v[2][NVMAX][W];
};

// Reduce NV sums over the whole cluster.  vals[k][a] is this thread's value
// for atom slot a; the result for k is tree_a( tree_w( wave_sum ) ), i.e. the
// pairwise sum over the atom index i = a*T + w*64 + lane padded to a power of
// two.  Every thread of the team receives every result.
template <int W, int A, int NV, int NVMAX, int L = kWave>
__device__ __forceinline__ void team_sum(double (&vals)[NV][A], double (&out)[NV],
                                         TeamScratch<W, NVMAX>& sc, int& bank) {
    static_assert(NV * A <= NVMAX, "scratch too small");
    static_assert(L == kWave || (W == 1 && A == 1), "16 leaves: one wavefront, one slot");
    double ws[NV][A];
#pragma unroll
    for (int a = 0; a < A; ++a) {
        if constexpr (NV == 4) {
            double o4[4];
            wave_sum4(vals[0][a], vals[1][a], vals[2][a], vals[3][a], o4);
#pragma unroll
            for (int k = 0; k < 4; ++k) ws[k][a] = o4[k];
        } else {
#pragma unroll
            for (int k = 0; k < NV; ++k) ws[k][a] = wave_sum<L>(vals[k][a]);
        }
    }
    if constexpr (W == 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double r[A];
#pragma unroll
            for (int a = 0; a < A; ++a) r[a] = ws[k][a];
            out[k] = tree<A>(r);
        }
    } else {
        const int w = threadIdx.x / kWave;
        const int lane = threadIdx.x % kWave;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k)
#pragma unroll
                for (int a = 0; a < A; ++a) sc.v[bank][k * A + a][w] = ws[k][a];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double r[A];
#pragma unroll
            for (int a = 0; a < A; ++a) {
                double rw[W];
#pragma unroll
                for (int q = 0; q < W; ++q) rw[q] = sc.v[bank][k * A + a][q];
                r[a] = tree_w<W>(rw);
            }
            out[k] = uniform(tree<A>(r));  // identical in every lane
        }
        bank ^= 1;
    }
}

template <int W, int A, int NVMAX, int L = kWave>
__device__ __forceinline__ double team_max(const double (&vals)[A], TeamScratch<W, NVMAX>& sc,
                                           int& bank) {
    double m = vals[0];
#pragma unroll
    for (int a = 1; a < A; ++a) m = fmax(m, vals[a]);
    m = wave_max<L>(m);
    if constexpr (W == 1) {
        return m;
    } else {
        const int w = threadIdx.x / kWave;
        if (threadIdx.x % kWave == 0) sc.v[bank][0][w] = m;
        __syncthreads();
        double r = sc.v[bank][0][0];
#pragma unroll
        for (int q = 1; q < W; ++q) r = fmax(r, sc.v[bank][0][q]);
        bank ^= 1;
        return uniform(r);
    }
}

// ---------------------------------------------------------------------------
// exp(z) by Cody-Waite reduction z = k ln2 + r (ln2 split into a high part
// of 32 significant bits, 21 trailing zero bits, so k ln2_hi is exact for
// |k| < 2^21, and a low part: the published split of fdlibm's e_exp.c,
// Sun 1993) and the degree-13 Taylor
// polynomial of e^r in Horner form (|r| <= ln2/2, truncation error below
// 2^-53), scaled by 2^k; 0 below -708 and for NaN.  Every operation is a
// correctly rounded IEEE operation, so the result does not depend on the
// device.  Used by the Metropolis test (z <= 0) and the Morse pair (z <= rho;
// the reduction and polynomial hold up to z = 709).
__device__ __forceinline__ double exp_cw(double z) {
    if (!(z >= -708.0)) return 0.0;
    const double kf = rint(z * 1.4426950408889634);
    double r = fma(-kf, 6.93147180369123816490e-01, z);
    r = fma(-kf, 1.90821492927058770002e-10, r);
    double p = 1.0 / 6227020800.0;
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

// ---------------------------------------------------------------------------
// Eq. (1) pair loops.  pos holds the cluster's coordinates in LDS as
// (x, y, z, pad); every lane reads the same partner j (LDS broadcast).
// Per atom i: e_i = sum_{j != i, ascending j} (s6^2 - s6) with q = 1/r^2,
// s6 = q^3, and g_i = sum_{j != i} q s6 (24 - 48 s6) (x_i - x_j).
// ---------------------------------------------------------------------------

// 1/x for 2^-767 <= x < 2^1022 with the operations of the IEEE division
// 1.0 / x that survive in that range: the hardware reciprocal estimate, two
// Newton steps y <- y + y (1 - x y), and the final correction
// q = y + y (1 - x y).  There the division's operand scaling (v_div_scale) is
// the identity and its special-case fix-up (v_div_fixup) returns q unchanged,
// so q is the same correctly rounded quotient.  For smaller x the pair term
// s6 = q^3 overflows in both forms (the energy is not finite) and for larger x
// both give s6 = 0; a non-finite energy is recomputed with the IEEE division.
__device__ __forceinline__ double recip_in_range(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(fma(-x, y, 1.0), y, y);
}

// One ordered pair (i = slot a of this thread, partner j at p), FP64.  The
// self pair (r2 = 0) adds exactly zero.  IEEE: q = 1 / r2 by
// the full division; otherwise recip_in_range (the same bits wherever the
// cluster's energy is finite).
template <bool IEEE>
__device__ __forceinline__ void pair_fp64(const double4 p, bool self, double xi, double yi,
                                          double zi, double k24, double km48, double& e,
                                          double& gx, double& gy, double& gz) {
    const double dx = xi - p.x;
    const double dy = yi - p.y;
    const double dz = zi - p.z;
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    // the self pair (r2 = 0) clears the high word of q: q is then zero or
    // subnormal, s6 = q^3 is exactly 0 and the pair adds exact zeros (one
    // select instead of two)
    double q = IEEE ? 1.0 / r2 : recip_in_range(r2);
    int2 qb = *reinterpret_cast<int2*>(&q);
    qb.y = self ? 0 : qb.y;
    q = *reinterpret_cast<double*>(&qb);
    const double s6 = (q * q) * q;
    e = e + fma(s6, s6, -s6);
    const double f = (q * s6) * fma(km48, s6, k24);  // k24 = 24, km48 = -48
    gx = fma(f, dx, gx);
    gy = fma(f, dy, gy);
    gz = fma(f, dz, gz);
}

__device__ __forceinline__ void pair_fp32(const float4 p, bool self, float xi, float yi, float zi,
                                          float& e, float& gx, float& gy, float& gz) {
    const float dx = xi - p.x;
    const float dy = yi - p.y;
    const float dz = zi - p.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float q = self ? 0.0f : __builtin_amdgcn_rcpf(r2);
    const float s6 = (q * q) * q;
    e = e + fmaf(s6, s6, -s6);
    const float f = (q * s6) * fmaf(-48.0f, s6, 24.0f);
    gx = fmaf(f, dx, gx);
    gy = fmaf(f, dy, gy);
    gz = fmaf(f, dz, gz);
}

// Morse pair (reduced units: well depth 1 at r = 1, range rho):
// V = t (t - 2), t = exp(rho (1 - r)); the gradient coefficient is
// (dV/dr) / r = ((c t) (t - 1)) / r with c = -2 rho.  Per atom i the partner
// sums are e_i = sum V and g_i = sum coefficient (x_i - x_j); E = 0.5 sum e_i.
// The self pair contributes exactly zero.
constexpr int kPairLJ = LJ_PAIR_LJ;
constexpr int kPairMorse = LJ_PAIR_MORSE;

__device__ __forceinline__ void pair_morse64(const double4 p, bool self, double xi, double yi,
                                             double zi, double rho, double c, double& e,
                                             double& gx, double& gy, double& gz) {
    const double dx = xi - p.x;
    const double dy = yi - p.y;
    const double dz = zi - p.z;
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const double r = sqrt(r2);
    const double t = self ? 0.0 : exp_cw(fma(-rho, r, rho));
    e = e + t * (t - 2.0);
    const double fn = (c * t) * (t - 1.0);
    const double f = self ? 0.0 : fn / r;
    gx = fma(f, dx, gx);
    gy = fma(f, dy, gy);
    gz = fma(f, dz, gz);
}

// The FP64 Morse terms of one distinct pair, with the operations of
// pair_morse64: .y = V and .x = the gradient coefficient, functions of r2
// alone.
__device__ __forceinline__ double2 term_morse64(double dx, double dy, double dz, double rho,
                                                double c) {
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const double r = sqrt(r2);
    const double t = exp_cw(fma(-rho, r, rho));
    const double et = t * (t - 2.0);
    const double fn = (c * t) * (t - 1.0);
    return make_double2(fn / r, et);
}

// FP32: hardware square root, base-2 exponential and reciprocal.
__device__ __forceinline__ void pair_morse32(const float4 p, bool self, float xi, float yi,
                                             float zi, float rho, float c, float& e, float& gx,
                                             float& gy, float& gz) {
    const float dx = xi - p.x;
    const float dy = yi - p.y;
    const float dz = zi - p.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float r = __builtin_amdgcn_sqrtf(r2);
    const float t = self ? 0.0f : __builtin_amdgcn_exp2f(fmaf(-rho, r, rho) * 1.44269504f);
    const float q = self ? 0.0f : __builtin_amdgcn_rcpf(r);
    e = e + t * (t - 2.0f);
    const float f = ((c * t) * (t - 1.0f)) * q;
    gx = fmaf(f, dx, gx);
    gy = fmaf(f, dy, gy);
    gz = fmaf(f, dz, gz);
}

// FP64: every operation rounded as written; partners are consumed in
// ascending order, so each per-atom sum is reproducible.  Partner
// coordinates are read from LDS in groups of kGroup64 ahead of the
// arithmetic to cover the LDS latency.
constexpr int kGroup64 = 4;
constexpr int kGroup32 = 8;

// t: the atom index of this thread's slot 0 (atom a T + t is slot a).
template <int A, int T, int POT, bool IEEE = true>
__device__ __forceinline__ void pairs_fp64(int n, const double4* __restrict__ pos,
                                           const double (&x)[3][A], double (&e)[A],
                                           double (&g)[3][A], double rho, int t) {
    const double c = -2.0 * rho;
    // 24 and -48 held in registers for the whole loop: a 64-bit constant that
    // is not an inline one would otherwise be rebuilt by two moves per pair
    double k24 = 24.0, km48 = -48.0;
    asm volatile("" : "+v"(k24));
    asm volatile("" : "+s"(km48));
    auto pair = [&](const double4 p, bool self, int a) {
        if constexpr (POT == kPairMorse)
            pair_morse64(p, self, x[0][a], x[1][a], x[2][a], rho, c, e[a], g[0][a], g[1][a],
                         g[2][a]);
        else
            pair_fp64<IEEE>(p, self, x[0][a], x[1][a], x[2][a], k24, km48, e[a], g[0][a],
                            g[1][a], g[2][a]);
    };
#pragma unroll
    for (int a = 0; a < A; ++a) {
        e[a] = 0.0;
        g[0][a] = g[1][a] = g[2][a] = 0.0;
    }
    int j = 0;
    for (; j + kGroup64 <= n; j += kGroup64) {
        double4 p[kGroup64];
#pragma unroll
        for (int u = 0; u < kGroup64; ++u) p[u] = pos[j + u];
#pragma unroll
        for (int u = 0; u < kGroup64; ++u)
#pragma unroll
            for (int a = 0; a < A; ++a) pair(p[u], j + u == a * T + t, a);
    }
    for (; j < n; ++j) {
        const double4 p = pos[j];
#pragma unroll
        for (int a = 0; a < A; ++a) pair(p, j == a * T + t, a);
    }
}

// FP64 Morse pair, one wavefront, one atom per lane (lane t holds atom t):
// every unique pair's terms once, then the oracle's ordered sums.  A Morse
// term (an exponential, a square root and a division) costs far more than
// the matrix's LDS traffic; the cheaper terms of Eq. (1) stay in the ordered
// loop, which is as fast for them.
//   1. The n (n - 1) / 2 unique pairs, listed once per cluster by
//      up_pair_list, go to the lanes in turn, 64 at a time.  Each pair's
//      (f, e term) is written to both slots M[i n + j] and M[j n + i] of an
//      n x n LDS matrix; the diagonal holds zeros.
//   2. Lane i adds M[j n + i] for j = 0 .. n - 1 in ascending order into
//      e_i and g_i = sum f (x_i - x_j), with x_i - x_j formed as in the
//      ordered loop.
// The terms depend on r2 only, which is the same from either side of a pair,
// so every sum sees the same terms in the same order as pairs_fp64: the
// results are bitwise equal, for half the pair terms.

// The pair list: entry p = (k - 1) n + i (ring order: atom i and partner
// (i + k) mod n, k = 1 .. n / 2; for even n the last distance on i < n / 2
// only) holds the byte offsets of both atoms in pos (x) and of both matrix
// slots (y), 16 bits each.  (p + 1/2) / n is at least 1 / (2 n) away from an
// integer, far more than the FP32 rounding of the product for p < 2^12, so
// its truncation is p / n exactly.  One wavefront; n <= 64.
__device__ __forceinline__ void up_pair_list(int n, uint2* __restrict__ list, int t) {
    const int P = n * (n - 1) / 2;
    if (P <= 0) return;
    const float inv_n = 1.0f / (float)n;
    for (int p = t; p < P; p += kWave) {
        const int k1 = (int)(((float)p + 0.5f) * inv_n);  // k - 1
        const int i = p - k1 * n;
        int j = i + k1 + 1;
        j = j >= n ? j - n : j;
        list[p] = make_uint2((uint32_t)(i * 32) | ((uint32_t)(j * 32) << 16),
                             (uint32_t)((i * n + j) * 16) | ((uint32_t)((j * n + i) * 16) << 16));
    }
}

constexpr int kUpRounds = 4;

__device__ __forceinline__ void pairs_morse64_up(int n, const double4* __restrict__ pos,
                                                 double2* __restrict__ M,
                                                 const uint2* __restrict__ list,
                                                 const double (&x)[3][1], double (&e)[1],
                                                 double (&g)[3][1], double rho, int t) {
    const double c = -2.0 * rho;
    const int P = n * (n - 1) / 2;
    const char* pb = reinterpret_cast<const char*>(pos);
    char* mb = reinterpret_cast<char*>(M);
    if (t < n) M[t * n + t] = make_double2(0.0, 0.0);
    // kUpRounds rounds of 64 pairs at a time, so that their LDS reads and
    // arithmetic overlap; entries past the list repeat its last one and are
    // not stored
    const int R = (P + kWave - 1) / kWave;
    for (int r0 = 0; r0 < R; r0 += kUpRounds) {
        uint2 w[kUpRounds];
        double4 pi[kUpRounds], pj[kUpRounds];
        double2 tt[kUpRounds];
#pragma unroll
        for (int u = 0; u < kUpRounds; ++u) w[u] = list[min(t + kWave * (r0 + u), P - 1)];
#pragma unroll
        for (int u = 0; u < kUpRounds; ++u) {
            pi[u] = *reinterpret_cast<const double4*>(pb + (w[u].x & 0xffffu));
            pj[u] = *reinterpret_cast<const double4*>(pb + (w[u].x >> 16));
        }
#pragma unroll
        for (int u = 0; u < kUpRounds; ++u)
            tt[u] = term_morse64(pi[u].x - pj[u].x, pi[u].y - pj[u].y, pi[u].z - pj[u].z, rho, c);
#pragma unroll
        for (int u = 0; u < kUpRounds; ++u)
            if (t + kWave * (r0 + u) < P) {
                *reinterpret_cast<double2*>(mb + (w[u].y & 0xffffu)) = tt[u];
                *reinterpret_cast<double2*>(mb + (w[u].y >> 16)) = tt[u];
            }
    }
    __syncthreads();  // one wavefront: the matrix is complete
    e[0] = 0.0;
    g[0][0] = g[1][0] = g[2][0] = 0.0;
    const double xi = x[0][0], yi = x[1][0], zi = x[2][0];
    const double2* Mi = M + (t < n ? t : (n > 0 ? n - 1 : 0));  // lanes >= n: results unused
    auto acc = [&](const double4 p, const double2 tt) {
        const double dx = xi - p.x;
        const double dy = yi - p.y;
        const double dz = zi - p.z;
        e[0] = e[0] + tt.y;
        g[0][0] = fma(tt.x, dx, g[0][0]);
        g[1][0] = fma(tt.x, dy, g[1][0]);
        g[2][0] = fma(tt.x, dz, g[2][0]);
    };
    int j = 0;
    for (; j + kGroup64 <= n; j += kGroup64) {
        double4 p[kGroup64];
        double2 tt[kGroup64];
#pragma unroll
        for (int u = 0; u < kGroup64; ++u) {
            p[u] = pos[j + u];
            tt[u] = Mi[(j + u) * n];
        }
#pragma unroll
        for (int u = 0; u < kGroup64; ++u) acc(p[u], tt[u]);
    }
    for (; j < n; ++j) acc(pos[j], Mi[j * n]);
}

// FP32 pair arithmetic and FP32 accumulation over tiles of kTileJ partners;
// each tile's per-atom partial sums are added into FP64 accumulators.
template <int A, int T, int POT>
__device__ __forceinline__ void pairs_mixed(int n, const float4* __restrict__ pos,
                                            const double (&x)[3][A], double (&e)[A],
                                            double (&g)[3][A], double rho, int t) {
    const float rf = (float)rho, cf = -2.0f * rf;
    float xf[3][A];
#pragma unroll
    for (int a = 0; a < A; ++a) {
        e[a] = 0.0;
        g[0][a] = g[1][a] = g[2][a] = 0.0;
        xf[0][a] = (float)x[0][a];
        xf[1][a] = (float)x[1][a];
        xf[2][a] = (float)x[2][a];
    }
    for (int j0 = 0; j0 < n; j0 += kTileJ) {
        const int j1 = min(n, j0 + kTileJ);
        float te[A], tg[3][A];
#pragma unroll
        for (int a = 0; a < A; ++a) te[a] = tg[0][a] = tg[1][a] = tg[2][a] = 0.0f;
        auto pair = [&](const float4 p, bool self, int a) {
            if constexpr (POT == kPairMorse)
                pair_morse32(p, self, xf[0][a], xf[1][a], xf[2][a], rf, cf, te[a], tg[0][a],
                             tg[1][a], tg[2][a]);
            else
                pair_fp32(p, self, xf[0][a], xf[1][a], xf[2][a], te[a], tg[0][a], tg[1][a],
                          tg[2][a]);
        };
        int j = j0;
        for (; j + kGroup32 <= j1; j += kGroup32) {
            float4 p[kGroup32];
#pragma unroll
            for (int u = 0; u < kGroup32; ++u) p[u] = pos[j + u];
#pragma unroll
            for (int u = 0; u < kGroup32; ++u)
#pragma unroll
                for (int a = 0; a < A; ++a) pair(p[u], j + u == a * T + t, a);
        }
        for (; j < j1; ++j) {
            const float4 p = pos[j];
#pragma unroll
            for (int a = 0; a < A; ++a) pair(p, j == a * T + t, a);
        }
#pragma unroll
        for (int a = 0; a < A; ++a) {
            e[a] += (double)te[a];
            g[0][a] += (double)tg[0][a];
            g[1][a] += (double)tg[1][a];
            g[2][a] += (double)tg[2][a];
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 Eq. (1) over unique pairs for large clusters: 64-atom tiles, one per
// wavefront-lane set (tile tau = atoms 64 tau .. 64 tau + 63, owned by the
// thread that holds them: tau = a W + w).  The tile's coordinates are staged
// twice in LDS (pos[128 tau + l] = pos[128 tau + 64 + l] = atom 64 tau + l),
// so lane l reaches atom (l + k) mod 64 of a tile at an immediate offset.
//   - diagonal: lane l pairs with l + 1 .. l + 32 (mod 64) of its own tile,
//     distance 32 on lanes 0-31 only (every pair of the tile once), with the
//     rotating reaction accumulator below and a final exchange of halves;
//   - round t = 1 .. nt/2: tile tau pairs with tile J = tau + t (mod nt), every
//     pair once; for even nt the last round meets each tile pair from both
//     sides, so each side takes half of the 64 ring distances.  The reaction
//     on J's atom (l + k) accumulates in a register that is rotated one lane
//     per step (DPP wave_rol:1, folded into the add), so after the last
//     distance k lane l holds the reaction on J's atom (l + k) mod 64; it goes
//     to that atom's slot of the round's LDS buffer, and after the round's
//     barrier the owner of J adds it.  In a round every tile is the partner of
//     exactly one tile, so no two writers meet (no atomics) and all sums have a
//     fixed order.
// Atoms n .. 64 nt - 1 are padding placed 1e8 apart on the x axis: their
// pair terms underflow to exactly zero.  FP32 partial sums cover one tile
// pair (at most 64 terms) and are added into FP64.  e_i is returned in the
// ordered-pair convention of pairs_mixed (E = 2 sum e_i): a unique pair adds
// twice its term to the lane that evaluates it.
// ---------------------------------------------------------------------------
// One wavefront with two atom slots per lane (the 65-128-atom class beside
// larger ones) keeps the ordered loop: that kernel is at the register limit,
// and the tiles' staging registers cost more than their saved arithmetic.
template <int W, int A>
constexpr bool kUseTiles = W * A * kWave <= 2048 && !(W == 1 && A == 2);

// A tile evaluates 32 ring distances per atom within itself, against n
// partners per atom in the ordered loop: the tiles win above n = 32 (where a
// one-wavefront cluster of at most 43 atoms takes the ring instead).
__device__ __forceinline__ bool tiles_for(int n) { return n > kWave / 2; }

constexpr float kPadSpacing = 1.0e8f;

__device__ __forceinline__ float rol1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xF, 0xF, true));
}

// Lane l takes lane (l + 32) mod 64's value.
__device__ __forceinline__ float swap_half_lanes(float v, int lane) {
    const int b = __float_as_int(v);
    auto x = __builtin_amdgcn_permlane32_swap(b, b, false, false);  // {lower half, upper half}
    return __int_as_float(lane < kWave / 2 ? (int)x[1] : (int)x[0]);
}

__device__ __forceinline__ float4 tile_pad(int i) {
    return make_float4(kPadSpacing * (float)(1 + (i & 63)), 0.0f, 0.0f, 0.0f);
}

// Pairs of this lane's atom pi with partner-tile atoms (lane + k) mod 64 for
// k = k_begin .. k_begin + NSTEPS - 1 (base: the partner tile's doubled copy).
// Returns the reaction register, which then holds the reaction on partner
// atom (lane + k_begin + NSTEPS - 1) mod 64.
template <int NSTEPS>
__device__ __forceinline__ float3 tile_pair(const float4 pi, const float4* __restrict__ base,
                                            int lane, int k_begin, float& te, float& tx,
                                            float& ty, float& tz) {
    float rx = 0.0f, ry = 0.0f, rz = 0.0f;
    const float4* src = base + lane;
#pragma unroll 1
    for (int k0 = k_begin; k0 < k_begin + NSTEPS; k0 += kGroup32) {
        float4 p[kGroup32];
#pragma unroll
        for (int u = 0; u < kGroup32; ++u) p[u] = src[k0 + u];
#pragma unroll
        for (int u = 0; u < kGroup32; ++u) {
            const float dx = pi.x - p[u].x;
            const float dy = pi.y - p[u].y;
            const float dz = pi.z - p[u].z;
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float q = __builtin_amdgcn_rcpf(r2);
            const float s6 = (q * q) * q;
            te = te + fmaf(s6, s6, -s6);
            const float f = (q * s6) * fmaf(-48.0f, s6, 24.0f);
            tx = fmaf(f, dx, tx);
            ty = fmaf(f, dy, ty);
            tz = fmaf(f, dz, tz);
            // lane l's accumulator moves to lane l - 1 before each step, so it
            // follows partner atom l + k (at the first step it rotates zeros)
            rx = rol1(rx) - f * dx;
            ry = rol1(ry) - f * dy;
            rz = rol1(rz) - f * dz;
        }
    }
    return make_float3(rx, ry, rz);
}

// ---------------------------------------------------------------------------
// FP32 pair terms (Eq. (1) or the Morse pair) over unique pairs for
// one-wavefront clusters of kRingMin <= n <= 43 atoms: a ring of period n.
// Lane l holds atom l mod n (lanes n .. 63 are replicas) and pairs with atom
// (l + k) mod n for k = 1 .. n/2; for even n the distance n/2 is taken by the
// lanes whose atom is below n/2 only, so every unique pair is evaluated once
// by a real lane.
// The reaction on the partner accumulates in a register rotated one lane per
// step (wave_rol:1): lane l receives lane l + 1's sum, which followed atom
// (l + 1) mod n + k - 1 = l mod n + k, for every lane except 63, which wraps to
// lane 0.  That one wrong value enters at lane 63 and moves down one lane per
// step, so after K steps lanes 0 .. 63 - K are exact, and these include every
// real lane when K <= 64 - n.  Steps run in groups of kRingGroup, the last
// group stopping at K; the result on lane l is the reaction on atom
// (l + K) mod n, returned to its owner through LDS.  The coordinates are staged
// as pos[j] = atom j mod n for j < 64 + K.  FP32 sums cover at most K <= 21
// terms and are added into FP64.  e_i follows the ordered-pair convention of
// pairs_mixed, as in pairs_tiles.
// ---------------------------------------------------------------------------
constexpr int kRingGroup = 4;
constexpr int kRingMin = 20;  // below, the ordered loop is as fast (staging and readout)

// Steps of the ring for n atoms: the distances 1 .. n/2.
__device__ __forceinline__ int ring_steps(int n) { return n / 2; }
__device__ __forceinline__ bool ring_for(int n) {
    return n >= kRingMin && ring_steps(n) <= kWave - n;
}

template <bool LAST, int POT>
__device__ __forceinline__ void ring_group(const float4 pi, const float4* __restrict__ src,
                                           int k0, int K, bool upper, float rho, float c,
                                           float& te, float& tx, float& ty, float& tz,
                                           float& rx, float& ry, float& rz) {
    float4 p[kRingGroup];
#pragma unroll
    for (int u = 0; u < kRingGroup; ++u) p[u] = src[LAST ? min(k0 + u, K) : k0 + u];
#pragma unroll
    for (int u = 0; u < kRingGroup; ++u) {
        // the last group stops at distance K (uniform); distance n/2 on the
        // upper lanes adds nothing
        bool skip = false;
        if constexpr (LAST) {
            if (k0 + u > K) break;
            skip = k0 + u == K && upper;
        }
        const float dx = pi.x - p[u].x;
        const float dy = pi.y - p[u].y;
        const float dz = pi.z - p[u].z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        float ep, f;
        if constexpr (POT == kPairMorse) {
            const float r = __builtin_amdgcn_sqrtf(r2);
            float t = __builtin_amdgcn_exp2f(fmaf(-rho, r, rho) * 1.44269504f);
            float q = __builtin_amdgcn_rcpf(r);
            if (skip) t = q = 0.0f;
            ep = t * (t - 2.0f);
            f = ((c * t) * (t - 1.0f)) * q;
        } else {
            float q = __builtin_amdgcn_rcpf(r2);
            if (skip) q = 0.0f;
            const float s6 = (q * q) * q;
            ep = fmaf(s6, s6, -s6);
            f = (q * s6) * fmaf(-48.0f, s6, 24.0f);
        }
        te = te + ep;
        tx = fmaf(f, dx, tx);
        ty = fmaf(f, dy, ty);
        tz = fmaf(f, dz, tz);
        rx = rol1(rx) - f * dx;
        ry = rol1(ry) - f * dy;
        rz = rol1(rz) - f * dz;
    }
}

template <int POT>
__device__ __forceinline__ void pairs_ring(int n, const float4* __restrict__ pos,
                                           float* __restrict__ rbuf, double& e,
                                           double (&g)[3][1], double rho) {
    const int lane = threadIdx.x;  // one wavefront
    const int K = ring_steps(n);
    const int al = lane % n;
    const bool upper = (n % 2 == 0) && al >= K;
    const float rf = (float)rho, cf = -2.0f * rf;
    const float4 pi = pos[lane];
    const float4* src = pos + lane;
    float te = 0.0f, tx = 0.0f, ty = 0.0f, tz = 0.0f;
    float rx = 0.0f, ry = 0.0f, rz = 0.0f;
    int k0 = 1;
#pragma unroll 1
    for (; k0 + kRingGroup - 1 < K; k0 += kRingGroup)
        ring_group<false, POT>(pi, src, k0, K, upper, rf, cf, te, tx, ty, tz, rx, ry, rz);
    // the last group, with 1 .. kRingGroup of the distances (K >= 1)
    ring_group<true, POT>(pi, src, k0, K, upper, rf, cf, te, tx, ty, tz, rx, ry, rz);
    if (lane < n) {  // lane l holds the reaction on atom (l + K) mod n, K < n
        int t = lane + K;
        if (t >= n) t -= n;
        rbuf[t] = rx;
        rbuf[kWave + t] = ry;
        rbuf[2 * kWave + t] = rz;
    }
    __syncthreads();
    e = 0.0;
    g[0][0] = g[1][0] = g[2][0] = 0.0;
    if (lane < n) {
        e = 2.0 * (double)te;
        g[0][0] = (double)tx + (double)rbuf[lane];
        g[1][0] = (double)ty + (double)rbuf[kWave + lane];
        g[2][0] = (double)tz + (double)rbuf[2 * kWave + lane];
    }
}

template <int W, int A>
__device__ __forceinline__ void pairs_tiles(int n, const float4* __restrict__ pos,
                                            float* __restrict__ rbuf, double (&e)[A],
                                            double (&g)[3][A]) {
    constexpr int T = kWave * W;
    constexpr int S = T * A;  // plane stride of the reaction buffer
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int nt = (n + kWave - 1) / kWave;
#pragma unroll
    for (int a = 0; a < A; ++a) {
        e[a] = 0.0;
        g[0][a] = g[1][a] = g[2][a] = 0.0;
        const int tau = a * W + w;
        if (tau >= nt) continue;
        const float4 pi = pos[128 * tau + lane];
        const float4* src = pos + 128 * tau + lane;
        float te = 0.0f, tx = 0.0f, ty = 0.0f, tz = 0.0f;
        float rx = 0.0f, ry = 0.0f, rz = 0.0f;
#pragma unroll 1
        for (int k0 = 1; k0 <= kWave / 2; k0 += kGroup32) {  // ring distances 1 .. 32
            float4 p[kGroup32];
#pragma unroll
            for (int u = 0; u < kGroup32; ++u) p[u] = src[k0 + u];
#pragma unroll
            for (int u = 0; u < kGroup32; ++u) {
                const float dx = pi.x - p[u].x;
                const float dy = pi.y - p[u].y;
                const float dz = pi.z - p[u].z;
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const float q = __builtin_amdgcn_rcpf(r2);
                // distance 32 pairs lanes l and l + 32: lanes 0-31 take it
                const bool dup = (u == kGroup32 - 1) && k0 + u == kWave / 2 && lane >= kWave / 2;
                const float s6 = dup ? 0.0f : (q * q) * q;
                te = te + fmaf(s6, s6, -s6);
                const float f = (q * s6) * fmaf(-48.0f, s6, 24.0f);
                tx = fmaf(f, dx, tx);
                ty = fmaf(f, dy, ty);
                tz = fmaf(f, dz, tz);
                rx = rol1(rx) - f * dx;
                ry = rol1(ry) - f * dy;
                rz = rol1(rz) - f * dz;
            }
        }
        // lane l now holds the reaction on atom l + 32: swap the two halves
        const float3 r = make_float3(swap_half_lanes(rx, lane), swap_half_lanes(ry, lane),
                                     swap_half_lanes(rz, lane));
        e[a] += 2.0 * (double)te;
        g[0][a] += (double)tx;
        g[1][a] += (double)ty;
        g[2][a] += (double)tz;
        g[0][a] += (double)r.x;
        g[1][a] += (double)r.y;
        g[2][a] += (double)r.z;
    }
    const int rounds = nt / 2;
    for (int t = 1; t <= rounds; ++t) {
        // For even nt the last round meets every tile pair from both sides:
        // tile tau < nt/2 takes ring distances 0 .. 31 towards its partner and
        // the partner takes distances 1 .. 32 back (distances 32 .. 63 seen
        // from tau), so both halves of the team work 32 steps.
        const bool half = (nt % 2 == 0) && t == rounds;
        float* rb = rbuf + (t & 1) * 3 * S;
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const int tau = a * W + w;
            if (tau >= nt) continue;
            int J = tau + t;
            if (J >= nt) J -= nt;
            const float4 pi = pos[128 * tau + lane];
            float te = 0.0f, tx = 0.0f, ty = 0.0f, tz = 0.0f;
            float3 r;
            int k_last;
            if (half) {
                const int k_begin = tau < rounds ? 0 : 1;
                r = tile_pair<kWave / 2>(pi, pos + 128 * J, lane, k_begin, te, tx, ty, tz);
                k_last = k_begin + kWave / 2 - 1;
            } else {
                r = tile_pair<kWave>(pi, pos + 128 * J, lane, 0, te, tx, ty, tz);
                k_last = kWave - 1;
            }
            e[a] += 2.0 * (double)te;
            g[0][a] += (double)tx;
            g[1][a] += (double)ty;
            g[2][a] += (double)tz;
            const int d = (lane + k_last) & (kWave - 1);  // the partner atom of the reaction
            rb[64 * J + d] = r.x;
            rb[S + 64 * J + d] = r.y;
            rb[2 * S + 64 * J + d] = r.z;
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < A; ++a) {  // every tile is the partner of exactly one tile
            const int tau = a * W + w;
            if (tau >= nt) continue;
            g[0][a] += (double)rb[64 * tau + lane];
            g[1][a] += (double)rb[S + 64 * tau + lane];
            g[2][a] += (double)rb[2 * S + 64 * tau + lane];
        }
    }
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128-bit multiplies; the key is bumped by the Weyl constants between
// rounds.
// ---------------------------------------------------------------------------
struct U64x4 {
    uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    U64x4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

constexpr uint64_t kPurposePerturb = 3;
constexpr uint64_t kPurposeMetropolis = 4;

// Top 53 bits of a random word as a double in [0, 1).
__device__ __forceinline__ double unit_double(uint64_t w) {
    return (double)(w >> 11) * 0x1.0p-53;
}

}  // namespace lj
