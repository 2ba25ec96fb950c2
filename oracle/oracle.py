"""numpy front end of the FP64 CPU oracle (oracle/lj_oracle.c).

TEST INFRASTRUCTURE ONLY.  Layouts follow the library boundary: coordinates
and gradients are three planes [3][total_atoms] (float64), clusters are
described by an int32 prefix-sum array offset[B+1].
"""
import ctypes as C

import numpy as np

from . import build as _build

CONVERGED, MAXITER, LSFAIL, NONFINITE = 0, 1, 2, 3

_lib = None


PAIRS = {"lj": 0, "morse": 1}


class LBFGSParams(C.Structure):
    _fields_ = [("m", C.c_int32), ("gtol", C.c_double), ("max_iter", C.c_int32),
                ("max_step", C.c_double), ("c1", C.c_double), ("max_ls", C.c_int32),
                ("curv_eps", C.c_double), ("pair", C.c_int32), ("rho", C.c_double)]


class BHParams(C.Structure):
    _fields_ = [("chains", C.c_int32), ("cands", C.c_int32), ("kT", C.c_double),
                ("adapt_interval", C.c_int32), ("target_rate", C.c_double),
                ("factor", C.c_double), ("seed", C.c_uint64)]


class ChainState(C.Structure):
    _fields_ = [("e_cur", C.c_double), ("step", C.c_double), ("win_accepts", C.c_int32),
                ("step_index", C.c_int64), ("e_best_seen", C.c_double),
                ("e_best_acc", C.c_double)]


class Trace(C.Structure):
    _fields_ = [("e_trial", C.c_void_p), ("accepted", C.c_void_p), ("e_best", C.c_void_p),
                ("e_best_acc", C.c_void_p), ("e_cur", C.c_void_p), ("step", C.c_void_p),
                ("ecand", C.c_void_p), ("cap", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(_build.ensure_built())
        d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        _lib.lj_o_tree_sum.restype = d
        _lib.lj_o_tree_sum.argtypes = [vp, i64]
        _lib.lj_o_energy_grad_batch.argtypes = [i32, vp, i64, vp, vp, vp, i32, d]
        _lib.lj_o_abs_sums_batch.argtypes = [i32, vp, i64, vp, vp, vp, i32, d]
        _lib.lj_o_minimize_batch.argtypes = [i32, vp, i64, vp, C.POINTER(LBFGSParams), vp, vp,
                                             vp, vp, vp]
        _lib.lj_o_two_loop.argtypes = [C.c_int, C.c_int, vp, vp, vp, d, vp, vp]
        _lib.lj_o_philox4x64_10.argtypes = [vp, vp, vp]
        _lib.lj_o_exp_bh.restype = d
        _lib.lj_o_exp_bh.argtypes = [d]
        _lib.lj_o_perturb.argtypes = [C.c_int, vp, d, C.c_uint64, i64, i64, i64, vp]
        _lib.lj_o_bh_decide.restype = C.c_int
        _lib.lj_o_bh_decide.argtypes = [C.POINTER(ChainState), C.POINTER(BHParams), i64, vp,
                                        C.POINTER(i32), C.POINTER(i32), C.POINTER(d)]
        _lib.lj_o_bh_run.argtypes = [i32, vp, i64, vp, vp, C.POINTER(ChainState),
                                     C.POINTER(BHParams), C.POINTER(LBFGSParams), i32,
                                     C.POINTER(Trace), i32]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def lbfgs_params(m=10, gtol=1e-6, max_iter=10000, max_step=0.2, c1=1e-4, max_ls=30,
                 curv_eps=1e-10, pair="lj", rho=6.0):
    return LBFGSParams(m, gtol, max_iter, max_step, c1, max_ls, curv_eps, PAIRS[pair], rho)


def tree_sum(v):
    v = _f64(v)
    return lib().lj_o_tree_sum(_p(v), v.size)


def energy_grad(offset, xyz, pair="lj", rho=6.0):
    """E[B] and gradient planes [3][T] of every cluster (Eq. 1 and its
    derivative, or the Morse pair of range rho)."""
    offset, xyz = _i32(offset), _f64(xyz)
    B, T = offset.size - 1, xyz.shape[-1]
    E = np.empty(B)
    g = np.empty((3, T))
    lib().lj_o_energy_grad_batch(B, _p(offset), T, _p(xyz), _p(E), _p(g), PAIRS[pair], rho)
    return E, g


def abs_sums(offset, xyz, pair="lj", rho=6.0):
    offset, xyz = _i32(offset), _f64(xyz)
    B, T = offset.size - 1, xyz.shape[-1]
    eabs = np.empty(B)
    gabs = np.empty((3, T))
    lib().lj_o_abs_sums_batch(B, _p(offset), T, _p(xyz), _p(eabs), _p(gabs), PAIRS[pair], rho)
    return eabs, gabs


def minimize(offset, xyz, params=None):
    """L-BFGS to ||g|| < gtol for every cluster; returns a dict of results."""
    params = params or lbfgs_params()
    offset = _i32(offset)
    x = _f64(xyz).copy()
    B, T = offset.size - 1, x.shape[-1]
    E, gn = np.empty(B), np.empty(B)
    it, ev, st = (np.empty(B, np.int32) for _ in range(3))
    lib().lj_o_minimize_batch(B, _p(offset), T, _p(x), C.byref(params), _p(E), _p(gn), _p(it),
                              _p(ev), _p(st))
    return dict(xyz=x, energy=E, gnorm=gn, iters=it, evals=ev, status=st)


def two_loop(S, Y, rho, gamma, g):
    """L-BFGS direction d = -H g from pairs S, Y ([hist][3][n], oldest first)."""
    S, Y, rho, g = _f64(S), _f64(Y), _f64(rho), _f64(g)
    hist, n = (S.shape[0], g.shape[-1]) if S.ndim == 3 else (0, g.shape[-1])
    d = np.empty((3, n))
    lib().lj_o_two_loop(n, hist, _p(S), _p(Y), _p(rho), float(gamma), _p(g), _p(d))
    return d


def philox4x64_10(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint64)
    key = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.empty(4, np.uint64)
    lib().lj_o_philox4x64_10(_p(ctr), _p(key), _p(out))
    return out


def exp_bh(z):
    return lib().lj_o_exp_bh(float(z))


def perturb(xcur, s, seed, chain, step, cand):
    """Perturbed copy (planes [3][n]) of one cluster's coordinates."""
    xcur = _f64(xcur)
    n = xcur.shape[-1]
    out = np.empty((3, n))
    lib().lj_o_perturb(n, _p(xcur), float(s), int(seed), int(chain), int(step), int(cand),
                       _p(out))
    return out


def bh_params(chains, cands, kT=0.8, adapt_interval=10, target_rate=0.5, factor=0.9, seed=0):
    return BHParams(chains, cands, kT, adapt_interval, target_rate, factor, seed)


def chain_state(e_cur, step, win_accepts=0, step_index=0, e_best_seen=np.inf, e_best_acc=None):
    return ChainState(e_cur, step, win_accepts, step_index, e_best_seen,
                      e_cur if e_best_acc is None else e_best_acc)


def bh_decide(state, params, chain, ecand):
    """One select / Metropolis / adapt decision; returns (sel, accepted, improved, e_sel)."""
    ecand = _f64(ecand)
    acc, imp, esel = C.c_int32(), C.c_int32(), C.c_double()
    sel = lib().lj_o_bh_decide(C.byref(state), C.byref(params), int(chain), _p(ecand),
                               C.byref(acc), C.byref(imp), C.byref(esel))
    return sel, acc.value, imp.value, esel.value


def bh_run(coff, xcur, states, params, lparams, num_steps, cap=None, xbest=None, chain0=0):
    """FP64 basin hopping for every chain; updates xcur / xbest / states in place.

    Chain c draws the random streams of chain chain0 + c (a slice of a larger
    set of chains run on its own).  Returns the trace as a dict of
    [chains][cap] arrays (ecand: [chains][cap][cands]).
    """
    coff = _i32(coff)
    chains = coff.size - 1
    assert xcur.dtype == np.float64 and xcur.flags.c_contiguous
    if xbest is None:
        xbest = xcur.copy()
    cap = num_steps if cap is None else cap
    nc = params.cands
    tr = dict(e_trial=np.full((chains, cap), np.nan), accepted=np.zeros((chains, cap), np.int8),
              e_best=np.full((chains, cap), np.nan), e_best_acc=np.full((chains, cap), np.nan),
              e_cur=np.full((chains, cap), np.nan), step=np.full((chains, cap), np.nan),
              ecand=np.full((chains, cap, nc), np.nan))
    t = Trace(*[tr[k].ctypes.data for k in ("e_trial", "accepted", "e_best", "e_best_acc",
                                             "e_cur", "step", "ecand")], cap)
    arr = (ChainState * chains)(*states)
    lib().lj_o_bh_run(chains, _p(coff), xcur.shape[-1], _p(xcur), _p(xbest), arr,
                      C.byref(params), C.byref(lparams), int(num_steps), C.byref(t), int(chain0))
    for c in range(chains):
        states[c] = arr[c]
    return tr
