"""The whole throughput-distortion GEMM, step by step (oracle; test infrastructure only).

C = A B with A (M x K) and B (K x N), following the paper's flow:

1. blocking into L x L subblocks (Sec. 2, eqs. 1-2) and per-block statistics
   (Sec. 3, Sec. 5.B)                                  -> ``blocks``
2. per-pair option records and, per inner kernel, pruning to the SNR budget
   (Sec. 5.B, Sec. 6)                                  -> ``control``
3. per pair: compand (eq. 3), pack (eqs. 6-7 or 11), packed product (eq. 8
   or 12), unpack (eqs. 9-10 or 13-14)                 -> ``packing``
4. reverse companding (eq. 5) and the l-sum of eq. (2), l ascending:
   C_ij = fma(r, inv, C_ij) for each pair, one rounding per pair (W = 1 pairs
   add their native product, i.e. inv = 1) -- an FMA chain over l; with
   k_groups > 1 the chain runs per group of consecutive l and the group sums
   are added in ascending order (eqs. 2 and 5 fix the sum, not its roundings).

Control modes:
* 'snr'        Sec. 5.B / Sec. 6 distortion control with a calibrated s(R, W).
* 'accel'      the same options pruned under the throughput constraint F_kernel (Sec. 6).
* 'fixed'      one (W, R_max) for every pair with the eq. (26) companders.
* 'separable'  per-block companders c = Q / max|X| with one Q and W.
* 'target'     one (W, R_max) for every pair with the Prop. 3 companders (eq. 22)
               that reach the expected subblock SNR snr_db.
'snr', 'accel' and 'target' take one target for all inner kernels or one per
inner kernel (S_kernel(i, j) or F_kernel(i, j), Sec. 6).

The result keeps every intermediate per pair when ``keep`` is set, indexed by
(i, j, l), plus the brute-force integer product of the companded blocks.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import blocks as bk
from . import control as ct
from . import packing as pk
from .fmachain import fma_matmul


@dataclass(frozen=True)
class Config:
    L: int = 64
    form: str = "sym"            # 'sym' (Sec. 3.B) or 'asym' (Sec. 3.C)
    prec: str = "f64"            # packing arithmetic: 'f64' or 'f32'
    ctrl: str = "snr"            # 'snr' | 'accel' | 'fixed' | 'separable' | 'target'
    snr_db: float = 40.0
    accel: float = 1.0           # 'accel': required fraction F_kernel of the maximum saved work
    # 'accel': saved-time units per W from measured accelerations F_W (Sec. 5.B),
    # as control.accel_units gives them; None counts nominal MFMA work
    accel_units: tuple | None = None
    # 'snr' / 'accel': optional per-inner-kernel targets, tile_targets[i][j] = S_kernel(i, j)
    # in dB or F_kernel(i, j) (Sec. 6); None uses snr_db / accel for every inner kernel
    tile_targets: tuple | None = None
    # evaluation order of the l-sum of eq. (2): k_groups groups of ceil(nL / k_groups)
    # consecutive subblocks, each summed from zero in ascending l, then the group sums
    # added in ascending order to zero (1: one ascending sum)
    k_groups: int = 1
    w_allowed: tuple = (1, 2)
    fixed_w: int = 2
    fixed_rmax: float = float(2 ** 20)
    sep_q: float = 127.0
    u_safe: float = 50.0


@dataclass
class Plan:
    cfg: Config
    M: int
    N: int
    K: int
    stats_a: list          # [i][l] BlockStats
    stats_b: list          # [l][j] BlockStats
    options: dict          # (i, j, l) -> {W: PairOption}
    chosen: dict           # (i, j, l) -> PairOption
    budget: dict           # (i, j) -> D_kernel ('snr' mode)

    @property
    def grid(self):
        L = self.cfg.L
        return bk.n_blocks(self.M, L), bk.n_blocks(self.K, L), bk.n_blocks(self.N, L)


def make_plan(A: np.ndarray, B: np.ndarray, cfg: Config, calib: dict | None = None,
              tiles=None) -> Plan:
    """Steps 1-2. ``calib`` maps W -> CalibTable (needed in 'snr' mode).
    ``tiles`` restricts the plan to a list of inner kernels (i, j)."""
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    L = cfg.L
    sa = bk.all_block_stats(A, L)
    sb = bk.all_block_stats(B, L)
    nI, nL, nJ = bk.n_blocks(M, L), bk.n_blocks(K, L), bk.n_blocks(N, L)
    w_desc = sorted(set(cfg.w_allowed), reverse=True)
    if 1 not in w_desc:
        raise ValueError("W = 1 must be allowed")
    if tiles is None:
        tiles = [(i, j) for i in range(nI) for j in range(nJ)]
    options, chosen, budget = {}, {}, {}
    for (i, j) in tiles:
        opts_l = []
        for l in range(nL):
            L_eff = bk.valid_extent(K, l, L)
            a, b = sa[i][l], sb[l][j]
            o = {}
            for W in w_desc:
                if W == 1:
                    o[W] = ct.option_native()
                elif cfg.ctrl in ("snr", "accel"):
                    o[W] = ct.best_option(W, L_eff, a, b, calib[W], cfg.u_safe)
                elif cfg.ctrl == "fixed":
                    o[W] = ct.fixed_option(W, L_eff, a, b, cfg.fixed_rmax, cfg.u_safe)
                elif cfg.ctrl == "separable":
                    o[W] = ct.separable_option(W, L_eff, a, b, cfg.sep_q, cfg.u_safe)
                elif cfg.ctrl == "target":
                    s_ij = cfg.snr_db if cfg.tile_targets is None else cfg.tile_targets[i][j]
                    s_rep = ct.table_s_at(calib[W], cfg.fixed_rmax, W) if W > 1 else 0.0
                    o[W] = ct.target_option(W, L_eff, a, b, cfg.fixed_rmax, s_rep, s_ij, cfg.u_safe)
                else:
                    raise ValueError(cfg.ctrl)
            opts_l.append(o)
            options[(i, j, l)] = o
        if cfg.ctrl == "snr":
            terms = [ct.signal_term(bk.valid_extent(K, l, L), sa[i][l], sb[l][j]) for l in range(nL)]
            s_ij = cfg.snr_db if cfg.tile_targets is None else cfg.tile_targets[i][j]
            dk = ct.kernel_budget(terms, s_ij)
            budget[(i, j)] = dk
            ws = ct.prune(opts_l, w_desc, dk)
        elif cfg.ctrl == "accel":
            f_ij = cfg.accel if cfg.tile_targets is None else cfg.tile_targets[i][j]
            units = None if cfg.accel_units is None else dict(cfg.accel_units)
            ws = ct.prune_accel(opts_l, w_desc, f_ij, units)
        else:
            ws = [cfg.fixed_w] * nL
        for l in range(nL):
            chosen[(i, j, l)] = opts_l[l][ws[l]]
    return Plan(cfg, M, N, K, sa, sb, options, chosen, budget)


@dataclass
class PairTrace:
    """Intermediates of one pair (kept when requested)."""
    qa: np.ndarray
    qb: np.ndarray
    abar: np.ndarray
    bbar: np.ndarray
    rbar: np.ndarray
    r: np.ndarray          # unpacked integers (or the native product for W = 1)
    r_exact: np.ndarray | None   # brute-force int64 product of qa, qb (W > 1)


@dataclass
class Result:
    plan: Plan
    C: np.ndarray
    traces: dict = field(default_factory=dict)


def pair_product(a: np.ndarray, b: np.ndarray, opt: ct.PairOption, cfg: Config,
                 keep: bool = False):
    """Step 3 for one pair: returns (r, inv, trace or None), whose contribution
    to C is r * inv (step 4); W = 1 gives the native product and inv = 1."""
    prec = cfg.prec
    dt = pk.DTYPES[prec]
    if opt.W == 1:
        a_ = np.asarray(a, dtype=dt)
        b_ = np.asarray(b, dtype=dt)
        r = pk.packed_product(a_, b_, prec)
        tr = PairTrace(a_, b_, a_, b_, r, r, None) if keep else None
        return r, dt(1.0), tr
    qa = pk.compand(a, opt.c_a, prec)
    qb = pk.compand(b, opt.c_b, prec)
    if cfg.form == "sym":
        abar = pk.pack_sym_a(qa, opt.W, opt.p, prec)
        bbar = pk.pack_sym_b(qb, opt.W, opt.p, prec)
        rbar = pk.packed_product(abar, bbar, prec)
        r = pk.unpack_sym(rbar, opt.p, prec)
    elif cfg.form == "asym":
        abar = pk.pack_asym_a(qa, opt.W, opt.p, prec)
        bbar = qb
        rbar = pk.packed_product(abar, bbar, prec)
        r = pk.unpack_asym(rbar, opt.W, opt.p, prec)
    else:
        raise ValueError(cfg.form)
    tr = None
    if keep:
        r_exact = qa.astype(np.int64) @ qb.astype(np.int64)
        tr = PairTrace(qa, qb, abar, bbar, rbar, r, r_exact)
    return np.asarray(r, dtype=dt), dt(opt.inv), tr


def fma_chain_sum(rs: list, invs: list, prec: str) -> np.ndarray:
    """Per output, acc = 0; for each pair in order: acc = fma(r, inv, acc) in prec,
    each step one correctly rounded fused multiply-add: the FMA-chain product of
    the row (r_0, r_1, ...) by the column (inv_0, inv_1, ...)."""
    L0, L1 = rs[0].shape
    n = len(rs)
    rows = np.ascontiguousarray(np.stack(rs).reshape(n, L0 * L1).T).reshape(L0 * L1, 1, n)
    cols = np.ascontiguousarray(np.broadcast_to(np.asarray(invs, dtype=rows.dtype).reshape(1, n, 1),
                                                (L0 * L1, n, 1)))
    return fma_matmul(rows, cols, prec).reshape(L0, L1)


def group_size(nl: int, k_groups: int) -> int:
    """Subblocks per group of the l-sum: ceil(nL / k_groups) (at least 1)."""
    if k_groups < 1:
        raise ValueError("k_groups must be >= 1")
    return max(1, -(-nl // k_groups))


def run(A: np.ndarray, B: np.ndarray, cfg: Config, calib: dict | None = None,
        tiles=None, keep: bool = False, plan: Plan | None = None) -> Result:
    """Steps 1-4 over the requested inner kernels (all by default)."""
    if plan is None:
        plan = make_plan(A, B, cfg, calib, tiles)
    L = cfg.L
    nI, nL, nJ = plan.grid
    M, N = plan.M, plan.N
    if tiles is None:
        tiles = [(i, j) for i in range(nI) for j in range(nJ)]
    dt = pk.DTYPES[cfg.prec]
    C = np.zeros((M, N), dtype=dt)
    res = Result(plan, C)
    size = group_size(nL, cfg.k_groups)
    for (i, j) in tiles:
        total = np.zeros((L, L), dtype=dt)
        for l0 in range(0, nL, size):
            rs, invs = [], []
            for l in range(l0, min(l0 + size, nL)):
                a = bk.block(A, i, l, L)
                b = bk.block(B, l, j, L)
                r, inv, tr = pair_product(a, b, plan.chosen[(i, j, l)], cfg, keep)
                rs.append(r)
                invs.append(inv)
                if keep:
                    res.traces[(i, j, l)] = tr
            acc = fma_chain_sum(rs, invs, cfg.prec)
            total = (total + acc).astype(dt)
        rows = min(L, M - i * L)
        cols = min(L, N - j * L)
        C[i * L:i * L + rows, j * L:j * L + cols] = total[:rows, :cols]
    return res


def snr_db(C_hat: np.ndarray, C_ref: np.ndarray) -> float:
    """Output SNR against a reference product: 10 log10(||C||^2 / ||C_hat - C||^2)."""
    ref = np.asarray(C_ref, dtype=np.float64)
    err = np.asarray(C_hat, dtype=np.float64) - ref
    e2 = float(np.sum(err * err))
    return float("inf") if e2 == 0.0 else 10.0 * np.log10(float(np.sum(ref * ref)) / e2)
