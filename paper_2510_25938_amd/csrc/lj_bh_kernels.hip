// Basin-hopping step kernels (Algorithm Overview, steps 1 and 3-5):
// perturbation of n copies of every chain's current structure, selection of
// the lowest candidate, the Metropolis test, the windowed step-size
// adaptation and the bookkeeping of the running lowest energies.
#include <hip/hip_runtime.h>

#include "lj_kernels.hpp"

namespace lj {

// Step 1.  One workgroup per (chain, candidate).  Coordinate k = 3 atom + dim
// (the paper's flattened order) takes word k mod 4 of Philox block k / 4 of
// the stream keyed (seed, 0) with counter (block, chain, step, purpose<<32 |
// candidate), and moves by s (2u - 1): uniform in a cube of side 2s.
// Thread 0 of each workgroup also writes the candidate's offset.
__global__ __launch_bounds__(64) void perturb_kernel(const int32_t* coff, int chains, int max_n,
                                                     int64_t total_chain, BhStateDev s, BhDev p,
                                                     double* xc, int32_t* cand_off) {
    const int cid = blockIdx.x;
    const int c = cid / p.cands;
    const int j = cid % p.cands;
    const int oc = coff[c];
    int n = coff[c + 1] - oc;
    if (n < 0 || n > max_n) n = 0;  // reported as LJ_BADSIZE by the plan kernel
    const int64_t total_c = total_chain * p.cands;
    const int64_t co = (int64_t)p.cands * oc + (int64_t)j * n;
    if (threadIdx.x == 0) {
        cand_off[cid] = (int32_t)co;
        if (cid == chains * p.cands - 1) cand_off[cid + 1] = (int32_t)total_c;
    }
    const uint64_t step = (uint64_t)s.step_index[c];
    const double sz = s.step[c];
    const uint64_t c3 = (kPurposePerturb << 32) | (uint64_t)j;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int k0 = 3 * a;
        const uint64_t b0 = (uint64_t)(k0 / 4);
        const U64x4 r0 = philox4x64_10(b0, (uint64_t)c, step, c3, p.seed, 0);
        U64x4 r1 = r0;
        if ((k0 + 2) / 4 != k0 / 4) r1 = philox4x64_10(b0 + 1, (uint64_t)c, step, c3, p.seed, 0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int k = k0 + d;
            const uint64_t w = (k / 4 == k0 / 4) ? r0.v[k % 4] : r1.v[k % 4];
            const double v = 2.0 * unit_double(w) - 1.0;
            xc[d * total_c + co + a] = fma(sz, v, s.xyz_cur[d * total_chain + oc + a]);
        }
    }
}

// Bookkeeping once the accepted structure is final (after its polish, if
// any): the current energy becomes the polished one, the best accepted energy
// is updated, and trace row k is written.  Returns whether the best accepted
// structure improved.
__device__ int finalize_chain(int c, BhStateDev s, BhDev p, const double* ecand, int sel, int acc,
                              const double* polish_e, const int32_t* polish_st, BhTraceDev tr) {
    int imp = 0;
    if (acc) {
        if (polish_e) s.e_cur[c] = polish_e[c];
        if (s.e_cur[c] < s.e_best_acc[c]) {
            s.e_best_acc[c] = s.e_cur[c];
            imp = 1;
        }
    }
    const int64_t k = s.step_index[c] - 1;
    if (k >= 0 && k < tr.cap) {
        const int64_t r = (int64_t)c * tr.cap + k;
        if (tr.e_trial) tr.e_trial[r] = sel >= 0 ? ecand[(int64_t)c * p.cands + sel] : __builtin_nan("");
        if (tr.accepted) tr.accepted[r] = (int8_t)acc;
        if (tr.e_best) tr.e_best[r] = s.e_best_seen[c];
        if (tr.e_best_acc) tr.e_best_acc[r] = s.e_best_acc[c];
        if (tr.e_cur) tr.e_cur[r] = s.e_cur[c];
        if (tr.step) tr.step[r] = s.step[c];
        if (tr.polish_status) tr.polish_status[r] = (int8_t)(acc && polish_st ? polish_st[c] : -1);
        if (tr.e_cand)
            for (int j = 0; j < p.cands; ++j)
                tr.e_cand[r * p.cands + j] = ecand[(int64_t)c * p.cands + j];
    }
    return imp;
}

// Steps 3-5.  One workgroup per chain; lane 0 takes the decisions, then the
// whole workgroup copies an accepted candidate into the current structure.
// dec[c] = selected candidate, dec[chains + c] = accepted flag.  With FIN
// (no polish follows) the same workgroup also does the final bookkeeping of
// the step, which otherwise runs in finalize_kernel after the polish.
template <bool FIN>
__global__ __launch_bounds__(64) void decide_kernel(const int32_t* coff, int chains, int max_n,
                                                    int64_t total_chain, BhStateDev s, BhDev p,
                                                    const double* xc, const double* ecand,
                                                    int32_t* dec, BhTraceDev tr) {
    __shared__ int sh_sel, sh_acc, sh_imp;
    const int c = blockIdx.x;
    if (threadIdx.x == 0) {
        const int64_t k = s.step_index[c];
        int sel = -1;
        double best = __builtin_inf();
        for (int j = 0; j < p.cands; ++j) {
            const double e = ecand[(int64_t)c * p.cands + j];
            if (e < best) {
                best = e;
                sel = j;
            }
        }
        int acc = 0;
        if (sel >= 0) {
            const double dE = best - s.e_cur[c];
            if (dE <= 0.0) {
                acc = 1;
            } else {
                const U64x4 r = philox4x64_10(0, (uint64_t)c, (uint64_t)k,
                                              kPurposeMetropolis << 32, p.seed, 0);
                if (unit_double(r.v[0]) < exp_cw(-dE / p.kT)) acc = 1;
            }
            if (best < s.e_best_seen[c]) s.e_best_seen[c] = best;
            if (acc) {
                s.e_cur[c] = best;
                s.win_accepts[c] += 1;
            }
        }
        const int64_t k1 = k + 1;
        s.step_index[c] = k1;
        if (k1 % p.adapt_interval == 0) {
            const double target = p.target_rate * (double)p.adapt_interval;
            const double won = (double)s.win_accepts[c];
            if (won > target)
                s.step[c] = s.step[c] / p.factor;
            else if (won < target)
                s.step[c] = s.step[c] * p.factor;
            s.win_accepts[c] = 0;
        }
        dec[c] = sel;
        dec[chains + c] = acc;
        sh_sel = sel;
        sh_acc = acc;
        sh_imp = FIN ? finalize_chain(c, s, p, ecand, sel, acc, nullptr, nullptr, tr) : 0;
    }
    __syncthreads();
    if (!sh_acc) return;
    const int oc = coff[c];
    const int n = coff[c + 1] - oc;
    if (n < 0 || n > max_n) return;
    const int64_t total_c = total_chain * p.cands;
    const int64_t co = (int64_t)p.cands * oc + (int64_t)sh_sel * n;
    for (int a = threadIdx.x; a < n; a += blockDim.x)
        for (int d = 0; d < 3; ++d) {
            const double v = xc[d * total_c + co + a];
            s.xyz_cur[d * total_chain + oc + a] = v;
            if (FIN && sh_imp) s.xyz_best[d * total_chain + oc + a] = v;
        }
}

// Final bookkeeping of a step whose accepted structure was polished in
// between (finalize_chain), then the best accepted structure is updated.
__global__ __launch_bounds__(64) void finalize_kernel(const int32_t* coff, int chains, int max_n,
                                                      int64_t total_chain, BhStateDev s, BhDev p,
                                                      const double* ecand, const int32_t* dec,
                                                      const double* polish_e,
                                                      const int32_t* polish_st, BhTraceDev tr) {
    __shared__ int sh_imp;
    const int c = blockIdx.x;
    if (threadIdx.x == 0)
        sh_imp = finalize_chain(c, s, p, ecand, dec[c], dec[chains + c], polish_e, polish_st, tr);
    __syncthreads();
    if (!sh_imp) return;
    const int oc = coff[c];
    const int n = coff[c + 1] - oc;
    if (n < 0 || n > max_n) return;
    for (int a = threadIdx.x; a < n; a += blockDim.x)
        for (int d = 0; d < 3; ++d)
            s.xyz_best[d * total_chain + oc + a] = s.xyz_cur[d * total_chain + oc + a];
}

hipError_t launch_perturb(const int32_t* coff, int chains, int max_n, int64_t total_chain,
                          BhStateDev s, BhDev p, double* xc, int32_t* cand_off, hipStream_t st) {
    hipLaunchKernelGGL(perturb_kernel, dim3(chains * p.cands), dim3(64), 0, st, coff, chains, max_n,
                       total_chain, s, p, xc, cand_off);
    return hipGetLastError();
}

hipError_t launch_decide(const int32_t* coff, int chains, int max_n, int64_t total_chain,
                         BhStateDev s, BhDev p, const double* xc, const double* ecand,
                         int32_t* dec, const BhTraceDev* fin, hipStream_t st) {
    if (fin)
        hipLaunchKernelGGL(decide_kernel<true>, dim3(chains), dim3(64), 0, st, coff, chains,
                           max_n, total_chain, s, p, xc, ecand, dec, *fin);
    else
        hipLaunchKernelGGL(decide_kernel<false>, dim3(chains), dim3(64), 0, st, coff, chains,
                           max_n, total_chain, s, p, xc, ecand, dec, BhTraceDev{});
    return hipGetLastError();
}

hipError_t launch_finalize(const int32_t* coff, int chains, int max_n, int64_t total_chain,
                           BhStateDev s, BhDev p, const double* ecand, const int32_t* dec,
                           const double* polish_e, const int32_t* polish_st, BhTraceDev tr,
                           hipStream_t st) {
    hipLaunchKernelGGL(finalize_kernel, dim3(chains), dim3(64), 0, st, coff, chains, max_n,
                       total_chain, s, p, ecand, dec, polish_e, polish_st, tr);
    return hipGetLastError();
}

}  // namespace lj
