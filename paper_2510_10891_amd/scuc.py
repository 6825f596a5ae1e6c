"""Seeded synthetic SCUC LP relaxations: the input generator.

Builds the LP relaxation of the three-binary security-constrained unit-commitment
model of Section II of the paper (logic constraints eq.(status), minimum up/down
eq.(minup/down), production limits eq.(power_limit), ramping eq.(ramp up/down),
system balance and PTDF security rows eq.(security), objective eq.(obj)) on a
random DC network, in the row-bounded LP form

    min c^T x + offset   s.t.  row_lo <= A x <= row_hi,   col_lo <= x <= col_hi,

which contains the paper's form eq.(lp) (A x >= theta) as the case row_hi = +inf.

Optionally applies the paper's instance-aware scaling (Section III-A): production
quantities are divided by eta^P and costs multiplied by eta^P / eta^C, so the
scaled optimum times eta^C is the original optimum.

This module only produces inputs. It holds none of the solver's arithmetic and is
imported by both the oracle tests and the GPU path; neither side's solver code
lives here. Every random draw comes from a numpy Generator seeded by the caller.

Recipe choices the paper leaves open (initial status, start-up/shut-down ramp
capacity, line limits, contingency choice) are documented on each helper.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Variable slots inside one hour: columns are ordered hour-major as [t][u, v, w, p][g].
U, V, W, P = 0, 1, 2, 3


@dataclass
class LP:
    """A row-bounded LP in CSR form (host arrays, FP64 values).

    ``row_lo``/``row_hi``/``col_lo``/``col_hi`` may hold +-inf; ``row_lo == row_hi``
    marks an equality row.
    """
    m: int
    n: int
    row_ptr: np.ndarray  # int64 [m+1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray      # float64 [nnz]
    row_lo: np.ndarray   # float64 [m]
    row_hi: np.ndarray   # float64 [m]
    col_lo: np.ndarray   # float64 [n]
    col_hi: np.ndarray   # float64 [n]
    c: np.ndarray        # float64 [n]
    obj_offset: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.m, self.n))

    def replace(self, **kw) -> "LP":
        return dataclasses.replace(self, **kw)


@dataclass(frozen=True)
class SCUCConfig:
    """Sizes of one synthetic SCUC instance."""
    n_bus: int
    n_line: int
    n_gen: int
    T: int
    n_monitored: int | None = None   # None: every line is monitored
    n_contingency: int = 0           # N-1 outages per monitored line, via LODF
    ptdf_drop: float = 0.0           # |PTDF| below this is dropped (0: keep all)
    name: str = ""


# The three single-instance workloads: a 30-bus case small enough for exhaustive CPU
# checks, a 2,000-bus case with 300 monitored lines x (1 + 10 outages), and a
# 13,500-bus case (the size of the paper's largest MATPOWER system) with
# 1,000 monitored lines x (1 + 20 outages).
SMALL = SCUCConfig(30, 41, 10, 24, None, 0, 0.0, "scuc-30bus-10gen-T24")
MEDIUM = SCUCConfig(2000, 3000, 500, 48, 300, 10, 1e-3, "scuc-2000bus-500gen-T48")
LARGE = SCUCConfig(13500, 20000, 4000, 36, 1000, 20, 1e-3, "scuc-13500bus-4000gen-T36")

# Parent instances of the batch cycle through five sizes (buses, lines, units, hours,
# monitored lines, outages per line).
BATCH_PARENTS = [
    SCUCConfig(30, 41, 10, 24, None, 0, 0.0, "batch-30bus"),
    SCUCConfig(100, 150, 25, 24, 40, 3, 1e-3, "batch-100bus"),
    SCUCConfig(300, 450, 75, 36, 60, 4, 1e-3, "batch-300bus"),
    SCUCConfig(600, 900, 150, 48, 100, 5, 1e-3, "batch-600bus"),
    SCUCConfig(1000, 1500, 250, 48, 150, 6, 1e-3, "batch-1000bus"),
]
PRESETS = {"small": SMALL, "medium": MEDIUM, "large": LARGE}


# ----------------------------------------------------------------------------- network

def random_network(rng: np.random.Generator, n_bus: int, n_line: int):
    """Random connected graph: a random recursive spanning tree plus uniform extra edges.

    Returns (from_bus, to_bus, reactance) with reactances drawn from U[0.05, 0.3] p.u.
    No self loops and no parallel lines.
    """
    if n_line < n_bus - 1:
        raise ValueError("a connected graph needs at least n_bus - 1 lines")
    max_edges = n_bus * (n_bus - 1) // 2
    if n_line > max_edges:
        raise ValueError("too many lines for a simple graph")
    child = np.arange(1, n_bus)
    parent = np.floor(rng.random(n_bus - 1) * child).astype(np.int64)
    edges = set(zip(np.minimum(parent, child).tolist(), np.maximum(parent, child).tolist()))
    fr = list(np.minimum(parent, child))
    to = list(np.maximum(parent, child))
    while len(fr) < n_line:
        a, b = rng.integers(0, n_bus, size=2)
        if a == b:
            continue
        a, b = (int(a), int(b)) if a < b else (int(b), int(a))
        if (a, b) in edges:
            continue
        edges.add((a, b))
        fr.append(a)
        to.append(b)
    x = rng.uniform(0.05, 0.3, size=n_line)
    return np.asarray(fr, np.int64), np.asarray(to, np.int64), x


class DCNetwork:
    """DC power-flow sensitivities with bus 0 as the slack.

    ``ptdf_rows(lines)`` returns the power transfer distribution factors of the
    given lines: entry [k, b] is the flow on line lines[k] per unit injected at bus
    b and withdrawn at the slack bus (column 0 is zero).
    """

    def __init__(self, fr, to, x, n_bus):
        self.fr, self.to, self.x, self.n_bus = fr, to, x, n_bus
        L = len(fr)
        self.b = 1.0 / x
        rows = np.concatenate([np.arange(L), np.arange(L)])
        cols = np.concatenate([fr, to])
        vals = np.concatenate([np.ones(L), -np.ones(L)])
        self.M = sp.csr_matrix((vals, (rows, cols)), shape=(L, n_bus))  # line-bus incidence
        B = (self.M.T @ sp.diags(self.b) @ self.M).tocsc()
        # B is symmetric positive definite: a minimum-degree ordering of B + B^T keeps the
        # factors sparse (an order of magnitude less fill than the default column ordering)
        self._lu = spla.splu(B[1:, 1:].tocsc(), permc_spec="MMD_AT_PLUS_A",
                             options=dict(SymmetricMode=True), diag_pivot_thresh=0.0)

    def ptdf_rows(self, lines: np.ndarray) -> np.ndarray:
        lines = np.asarray(lines, np.int64)
        # PTDF_S^T = B_r^{-1} M_{S,r}^T diag(b_S)  (B_r symmetric)
        rhs = (self.M[lines][:, 1:].T @ sp.diags(self.b[lines])).toarray()
        sol = self._lu.solve(rhs)
        out = np.zeros((len(lines), self.n_bus))
        out[:, 1:] = sol.T
        return out

    def flows(self, injection: np.ndarray) -> np.ndarray:
        """Line flows for a balanced bus injection vector (used by generator pins)."""
        theta = np.zeros(self.n_bus)
        theta[1:] = self._lu.solve(injection[1:])
        return self.b * (self.M @ theta)


# ----------------------------------------------------------------------------- instance

@dataclass
class SCUCData:
    """Physical parameters of one generated instance (unscaled, MW and $)."""
    cfg: SCUCConfig
    gen_bus: np.ndarray
    p_max: np.ndarray
    p_min: np.ndarray
    ramp: np.ndarray
    startup_cap: np.ndarray
    cost: np.ndarray
    startup_cost: np.ndarray
    min_up: np.ndarray
    min_down: np.ndarray
    demand: np.ndarray        # [T] system demand
    bus_share: np.ndarray     # [n_bus] Dirichlet(1) weights
    sec_coef: np.ndarray      # [S, G] generator coefficients of the hour-invariant security rows
    sec_const: np.ndarray     # [S] sum_b delta_lb * share_b (multiplied by D_t per hour)
    sec_limit: np.ndarray     # [S] F_l^c
    sec_label: np.ndarray     # [S, 2] (monitored line, outage line or -1)
    seed: int = 0
    sec_bus: sp.csr_matrix | None = None   # [S, n_bus] bus-level coefficients (full formulation)


def _draw_generators(rng, cfg: SCUCConfig):
    G = cfg.n_gen
    gen_bus = rng.integers(0, cfg.n_bus, size=G)
    p_max = rng.uniform(50.0, 300.0, size=G)
    cost = rng.uniform(10.0, 60.0, size=G)
    startup_cost = rng.uniform(100.0, 2000.0, size=G)
    min_up = rng.integers(1, 5, size=G)
    min_down = rng.integers(1, 5, size=G)
    return gen_bus, p_max, cost, startup_cost, min_up, min_down


def make_scuc_data(cfg: SCUCConfig, seed: int, bus_rows: bool = False) -> SCUCData:
    """Draw the network, generators, demand and the security rows of one instance.
    With ``bus_rows`` the bus-level coefficients of the kept security rows are stored as
    well (the full formulation puts the demand-penalty slack of every bus in them).

    Readings of details the recipe leaves open:
      * min production 0.3 p_max, ramp 0.5 p_max per hour, start-up and shut-down
        capacity SU = SD = max(p_min, ramp) = 0.5 p_max;
      * demand D_t = 0.6 sum(p_max) (1 + 0.25 sin(2 pi t / 24)), t = 1..T, split over
        buses by fixed Dirichlet(1) weights;
      * monitored lines: a seeded uniform sample; outages: a seeded sample of
        non-bridge lines (|1 - PTDF_kk| > 1e-6); post-outage PTDF rows by LODF;
      * line limits F = 1.2 max_t |flow| of the feasible dispatch
        p_gt = D_t p_max_g / sum(p_max) (all units on), floored at 1e-3 max F;
      * PTDF entries with |.| < ptdf_drop are dropped (bus level, before mapping to
        generators), and always those below 1e-10 (round-off of exact zeros); rows
        left with no generator coefficient are omitted.
    """
    rng = np.random.default_rng(seed)
    fr, to, x = random_network(rng, cfg.n_bus, cfg.n_line)
    net = DCNetwork(fr, to, x, cfg.n_bus)
    gen_bus, p_max, cost, startup_cost, min_up, min_down = _draw_generators(rng, cfg)
    share = rng.dirichlet(np.ones(cfg.n_bus))
    t = np.arange(1, cfg.T + 1)
    demand = 0.6 * p_max.sum() * (1.0 + 0.25 * np.sin(2.0 * np.pi * t / 24.0))

    L = cfg.n_line
    if cfg.n_monitored is None:
        monitored = np.arange(L)
    else:
        monitored = np.sort(rng.choice(L, size=min(cfg.n_monitored, L), replace=False))
    outages = np.zeros(0, np.int64)
    if cfg.n_contingency > 0:
        cand = rng.permutation(L)[: min(L, 4 * cfg.n_contingency + 8)]
        pc = net.ptdf_rows(cand)
        phi = pc[np.arange(len(cand)), fr[cand]] - pc[np.arange(len(cand)), to[cand]]
        ok = np.abs(1.0 - phi) > 1e-6
        outages = cand[ok][: cfg.n_contingency]
        if len(outages) < cfg.n_contingency:
            raise RuntimeError("not enough non-bridge lines for the requested outages")
        out_ptdf = pc[ok][: cfg.n_contingency]
        out_phi_self = phi[ok][: cfg.n_contingency]

    G = cfg.n_gen
    P_total = p_max.sum()
    coef_blocks, const_blocks, label_blocks, q_blocks, bus_blocks = [], [], [], [], []
    chunk = 256
    drop = max(cfg.ptdf_drop, 1e-10)   # entries that are zero in exact arithmetic come out as ~1e-17

    def reduce_block(D, lab):
        D[np.abs(D) < drop] = 0.0
        coef = D[:, gen_bus]                            # [k, G]
        const = D @ share
        keep = np.any(coef != 0.0, axis=1)
        q = coef @ p_max / P_total - const              # flow per unit demand of the feasible dispatch
        coef_blocks.append(coef[keep])
        const_blocks.append(const[keep])
        label_blocks.append(lab[keep])
        q_blocks.append(q[keep])
        if bus_rows:
            bus_blocks.append(sp.csr_matrix(D[keep]))

    for s0 in range(0, len(monitored), chunk):
        mon = monitored[s0:s0 + chunk]
        base = net.ptdf_rows(mon)                       # [k, n_bus]
        parts = [(base.copy(), np.stack([mon, -np.ones_like(mon)], 1))]
        for j, kline in enumerate(outages):
            # flow change on line l per unit transfer from->to of the outaged line
            phi_l = base[:, fr[kline]] - base[:, to[kline]]
            lodf = phi_l / (1.0 - out_phi_self[j])
            post = base + lodf[:, None] * out_ptdf[j][None, :]
            post[mon == kline] = 0.0                    # an outaged line carries no flow
            parts.append((post, np.stack([mon, np.full_like(mon, kline)], 1)))
        # rows in the order base case, outage 1, ..., outage C within the chunk
        for D, lab in parts:
            reduce_block(D, lab)
    sec_coef = np.concatenate(coef_blocks, 0) if coef_blocks else np.zeros((0, G))
    sec_const = np.concatenate(const_blocks) if const_blocks else np.zeros(0)
    sec_label = np.concatenate(label_blocks, 0) if label_blocks else np.zeros((0, 2), np.int64)
    q = np.concatenate(q_blocks) if q_blocks else np.zeros(0)
    F = 1.2 * demand.max() * np.abs(q)
    if len(F):
        F = np.maximum(F, 1e-3 * F.max())
    p_min = 0.3 * p_max
    ramp = 0.5 * p_max
    su = np.maximum(p_min, ramp)
    sec_bus = None
    if bus_rows:
        sec_bus = sp.vstack(bus_blocks, format="csr") if bus_blocks else sp.csr_matrix((0, cfg.n_bus))
    return SCUCData(cfg, gen_bus, p_max, p_min, ramp, su, cost, startup_cost, min_up, min_down,
                    demand, share, sec_coef, sec_const, F, sec_label, seed, sec_bus)


def col_index(G: int, t: int | np.ndarray, var: int, g: int | np.ndarray):
    """Column of variable ``var`` (U, V, W or P) of generator g in hour t (0-based)."""
    return np.asarray(t) * 4 * G + var * G + np.asarray(g)


def _csr_from_coo(nrows, r, cidx, v):
    order = np.lexsort((cidx, r))
    r, cidx, v = r[order], cidx[order], v[order]
    ptr = np.zeros(nrows + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=nrows), out=ptr[1:])
    return ptr, cidx.astype(np.int32), v.astype(np.float64)


def _status_rows(add, data: SCUCData, t: int, nrow: int, lo, hi, kind, KIND) -> int:
    """Rows of hour t on the commitment variables only, appended from local row `nrow` on:
    logic u_t - u_{t-1} - v_t + w_t = 0 (u_0 = 1 moves to the rhs at t = 1) and
    v_t + w_t <= 1 (eq.(status)), minimum up sum_{tau=max(1,t-UT+1)}^{t} v_tau - u_t <= 0 and
    minimum down sum w_tau + u_t <= 1 (eq.(minup/down)). Returns the next free local row."""
    G = data.cfg.n_gen
    g = np.arange(G)
    inf = np.inf
    # logic
    rr = nrow + g
    add(rr, col_index(G, t, U, g), np.ones(G))
    add(rr, col_index(G, t, V, g), -np.ones(G))
    add(rr, col_index(G, t, W, g), np.ones(G))
    if t >= 1:
        add(rr, col_index(G, t - 1, U, g), -np.ones(G))
        rhs = np.zeros(G)
    else:
        rhs = np.ones(G)
    lo.append(rhs); hi.append(rhs.copy()); kind.append(np.full(G, KIND["logic"]))
    nrow += G
    # v_t + w_t <= 1
    rr = nrow + g
    add(rr, col_index(G, t, V, g), np.ones(G))
    add(rr, col_index(G, t, W, g), np.ones(G))
    lo.append(np.full(G, -inf)); hi.append(np.ones(G)); kind.append(np.full(G, KIND["vw"]))
    nrow += G
    # min up
    rr = nrow + g
    add(rr, col_index(G, t, U, g), -np.ones(G))
    for d in range(int(data.min_up.max())):
        sel = (d < data.min_up) & (t - d >= 0)
        add(rr[sel], col_index(G, t - d, V, g[sel]), np.ones(int(sel.sum())))
    lo.append(np.full(G, -inf)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["min_up"]))
    nrow += G
    # min down
    rr = nrow + g
    add(rr, col_index(G, t, U, g), np.ones(G))
    for d in range(int(data.min_down.max())):
        sel = (d < data.min_down) & (t - d >= 0)
        add(rr[sel], col_index(G, t - d, W, g[sel]), np.ones(int(sel.sum())))
    lo.append(np.full(G, -inf)); hi.append(np.ones(G)); kind.append(np.full(G, KIND["min_dn"]))
    return nrow + G


def build_lp(data: SCUCData, instance_scaling: bool = True) -> LP:
    """Assemble the LP relaxation (rows hour by hour) from generated data.

    Rows of hour t, in order: balance; per generator: ramp up / ramp down (t >= 2),
    p - p_min u >= 0, p - p_max u <= 0, logic u_t - u_{t-1} - v_t + w_t = 0 (u_0 = 1 at t = 1),
    v_t + w_t <= 1, min-up window, min-down window; security (ranged) last. A unit's output column
    of hour t then meets rows from the start of hour t's block to the ramp rows near the start of
    hour t + 1's, so its column of A spans about one hour of rows (with the security rows first
    it spanned into the next hour's security block).
    With ``instance_scaling`` the production data are divided by eta^P = max p_max and
    costs scaled by eta^P/eta^C (production) and 1/eta^C (start-up), eta^C = max cost.
    """
    cfg = data.cfg
    G, T = cfg.n_gen, cfg.T
    if instance_scaling:
        eta_p = float(data.p_max.max())
        eta_c = float(data.cost.max())
    else:
        eta_p = eta_c = 1.0
    pmin = data.p_min / eta_p
    pmax = data.p_max / eta_p
    ru = data.ramp / eta_p
    su = data.startup_cap / eta_p
    dem = data.demand / eta_p
    F = data.sec_limit / eta_p
    n = 4 * G * T
    g = np.arange(G)

    # hour-invariant security block in CSR over generator index
    S = data.sec_coef.shape[0]
    nzr, nzc = np.nonzero(data.sec_coef)
    sec_ptr = np.zeros(S + 1, np.int64)
    np.cumsum(np.bincount(nzr, minlength=S), out=sec_ptr[1:])
    sec_gen = nzc.astype(np.int64)
    sec_val = data.sec_coef[nzr, nzc]

    ptr_parts, col_parts, val_parts, lo_parts, hi_parts = [], [], [], [], []
    row_kind_parts, row_hour_parts, row_sec_parts = [], [], []
    KIND = {"balance": 0, "security": 1, "lim_lo": 2, "lim_hi": 3, "ramp_up": 4,
            "ramp_dn": 5, "logic": 6, "vw": 7, "min_up": 8, "min_dn": 9}
    inf = np.inf
    for t in range(T):
        # balance
        ptr_parts.append(np.array([G], np.int64))
        col_parts.append(col_index(G, t, P, g).astype(np.int32))
        val_parts.append(np.ones(G))
        lo_parts.append(np.array([dem[t]]))
        hi_parts.append(np.array([dem[t]]))
        row_kind_parts.append(np.array([KIND["balance"]], np.int8))
        row_sec_parts.append(np.array([-1], np.int32))
        # generator rows, assembled as COO then sorted into CSR
        r_list, c_list, v_list, lo, hi, kind = [], [], [], [], [], []
        nrow = 0

        def add(rows_local, cols, vals):
            r_list.append(rows_local)
            c_list.append(cols)
            v_list.append(vals)

        if t >= 1:
            # p_t - p_{t-1} - RU u_{t-1} - SU v_t <= 0
            rr = nrow + g
            add(rr, col_index(G, t, P, g), np.ones(G))
            add(rr, col_index(G, t - 1, P, g), -np.ones(G))
            add(rr, col_index(G, t - 1, U, g), -ru)
            add(rr, col_index(G, t, V, g), -su)
            lo.append(np.full(G, -inf)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["ramp_up"]))
            nrow += G
            # p_{t-1} - p_t - RD u_t - SD w_t <= 0
            rr = nrow + g
            add(rr, col_index(G, t - 1, P, g), np.ones(G))
            add(rr, col_index(G, t, P, g), -np.ones(G))
            add(rr, col_index(G, t, U, g), -ru)
            add(rr, col_index(G, t, W, g), -su)
            lo.append(np.full(G, -inf)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["ramp_dn"]))
            nrow += G
        # p - pmin u >= 0
        rr = nrow + g
        add(rr, col_index(G, t, P, g), np.ones(G))
        add(rr, col_index(G, t, U, g), -pmin)
        lo.append(np.zeros(G)); hi.append(np.full(G, inf)); kind.append(np.full(G, KIND["lim_lo"]))
        nrow += G
        # p - pmax u <= 0
        rr = nrow + g
        add(rr, col_index(G, t, P, g), np.ones(G))
        add(rr, col_index(G, t, U, g), -pmax)
        lo.append(np.full(G, -inf)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["lim_hi"]))
        nrow += G
        nrow = _status_rows(add, data, t, nrow, lo, hi, kind, KIND)

        bptr, bcol, bval = _csr_from_coo(nrow, np.concatenate(r_list), np.concatenate(c_list),
                                         np.concatenate(v_list))
        ptr_parts.append(np.diff(bptr))
        col_parts.append(bcol)
        val_parts.append(bval)
        lo_parts.append(np.concatenate(lo))
        hi_parts.append(np.concatenate(hi))
        row_kind_parts.append(np.concatenate(kind).astype(np.int8))
        row_sec_parts.append(np.full(nrow, -1, np.int32))
        # security (ranged rows)
        if S:
            ptr_parts.append(np.diff(sec_ptr))
            col_parts.append(col_index(G, t, P, sec_gen).astype(np.int32))
            val_parts.append(sec_val)
            mid = data.sec_const * data.demand[t] / eta_p
            lo_parts.append(mid - F)
            hi_parts.append(mid + F)
            row_kind_parts.append(np.full(S, KIND["security"], np.int8))
            row_sec_parts.append(np.arange(S, dtype=np.int32))
        row_hour_parts.append(np.full(1 + S + nrow, t, np.int16))

    lens = np.concatenate(ptr_parts)
    row_ptr = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    col_idx = np.concatenate(col_parts).astype(np.int32)
    val = np.concatenate(val_parts).astype(np.float64)
    row_lo = np.concatenate(lo_parts)
    row_hi = np.concatenate(hi_parts)

    col_lo = np.zeros(n)
    col_hi = np.ones(n)
    # p <= p_max: implied by p - p_max u <= 0 and u <= 1 (the feasible set does not change);
    # stated as a column bound so that every column is boxed
    pcols = col_index(G, np.arange(T)[:, None], P, g[None, :]).ravel()
    col_hi[pcols] = np.tile(pmax, T)
    c = np.zeros(n)
    tt = np.arange(T)[:, None]
    c[col_index(G, tt, P, g[None, :]).ravel()] = np.tile(data.cost * eta_p / eta_c, T)
    c[col_index(G, tt, V, g[None, :]).ravel()] = np.tile(data.startup_cost / eta_c, T)

    meta = dict(config=cfg, G=G, T=T, eta_p=eta_p, eta_c=eta_c,
                row_kind=np.concatenate(row_kind_parts), row_kinds=KIND,
                row_hour=np.concatenate(row_hour_parts), row_sec=np.concatenate(row_sec_parts))
    return LP(len(lens), n, row_ptr, col_idx, val, row_lo, row_hi, col_lo, col_hi, c, 0.0, meta)


# ----------------------------------------------------------------------------- full formulation

# Unserved-demand penalty C^pen ($/MWh): well above every marginal cost of the recipe.
PEN_COST = 1000.0


def full_col_index(G: int, H: int, t: int | np.ndarray, slot: int, g: int | np.ndarray, T: int):
    """Column of an extra generator variable of the full formulation: slot 0 = p' (output
    above minimum), 1..H = segment outputs p_{gth}, H + 1 = production cost c_{gt}. The extras
    follow the 4 G T columns of the compact layout, which keep their positions, hour-major as
    [t][p', p_1..p_H, c][g]."""
    return 4 * G * T + (np.asarray(t) * (H + 2) + slot) * G + np.asarray(g)


def pen_col_index(G: int, H: int, T: int, n_bus: int, t: int | np.ndarray, b: int | np.ndarray):
    """Column of the unserved demand d^pen of bus b in hour t (after every generator column)."""
    return 4 * G * T + T * (H + 2) * G + np.asarray(t) * n_bus + np.asarray(b)


def segment_data(data: SCUCData, H: int):
    """Piecewise-linear production cost of eq.(prod_cost) (recipe readings): H segments of
    equal width splitting [P^L, P^U]; the first priced at the unit's cost, each next one dearer
    by a seeded factor U[1.05, 1.3] (a convex cost curve); no-load cost C^L = cost * P^L, the
    cost of running at P^L at the first segment's rate. Returns (width [G, H] MW,
    cost [G, H] $/MWh, no-load cost [G] $/h)."""
    rng = np.random.default_rng([data.seed, 1])
    G = data.cfg.n_gen
    width = np.repeat(((data.p_max - data.p_min) / H)[:, None], H, 1)
    steps = rng.uniform(1.05, 1.3, size=(G, H - 1))
    cost = data.cost[:, None] * np.concatenate([np.ones((G, 1)), np.cumprod(steps, 1)], 1)
    return width, cost, data.cost * data.p_min


def build_full_lp(data: SCUCData, instance_scaling: bool = True, segments: int = 3,
                  pen_cost: float = PEN_COST) -> LP:
    """The LP relaxation of the full model of Section II: output above minimum p', piecewise
    cost segments and cost variables (eq.(prod_cost)), no-load cost C^L u and unserved demand
    d^pen with penalty C^pen in the balance and security rows (eq.(security), eq.(obj)).

    The generator output p_gt of the balance and security rows is kept as a column, tied to
    the rest by p - p' - P^L u = 0 (so the security rows keep their PTDF coefficients);
    production limits, ramping (written in p' and u as in eq.(ramp up/down)) and the cost rows
    carry the capacity and cost parameters. Rows of hour t, in order: balance; security; per
    generator: definition of p, p' - (P^U - P^L) u <= 0, ramp up / down (t >= 2), H segment
    limits p_h - (P^U_h - P^U_{h-1}) u <= 0, sum_h p_h - p' = 0, sum_h C_h p_h - c = 0, then the
    commitment rows of the compact form. Start-up costs stay on v as in the compact form.
    Instance-aware scaling divides production data by eta^P = max P^U and multiplies costs by
    eta^P / eta^C with eta^C = the largest segment cost (Section III-A).
    """
    cfg = data.cfg
    G, T, B, H = cfg.n_gen, cfg.T, cfg.n_bus, segments
    S = data.sec_coef.shape[0]
    if S and data.sec_bus is None:
        raise ValueError("the full formulation needs the bus-level security rows "
                         "(make_scuc_data(..., bus_rows=True))")
    width, seg_cost, noload = segment_data(data, H)
    if instance_scaling:
        eta_p = float(data.p_max.max())
        eta_c = float(seg_cost.max())
    else:
        eta_p = eta_c = 1.0
    pmin = data.p_min / eta_p
    pmax = data.p_max / eta_p
    ru = data.ramp / eta_p
    su = data.startup_cap / eta_p
    wd = width / eta_p
    cs = seg_cost * eta_p / eta_c
    dem = data.demand / eta_p
    F = data.sec_limit / eta_p
    n = 4 * G * T + T * (H + 2) * G + T * B
    g = np.arange(G)
    bus = np.arange(B)

    # security rows over [generators | buses], hour-invariant
    sec = sp.hstack([sp.csr_matrix(data.sec_coef), data.sec_bus if S else sp.csr_matrix((0, B))],
                    format="csr")
    sec.sort_indices()
    sec_is_gen = sec.indices < G

    ptr_parts, col_parts, val_parts, lo_parts, hi_parts = [], [], [], [], []
    row_kind_parts, row_hour_parts, row_sec_parts = [], [], []
    KIND = {"balance": 0, "security": 1, "lim_lo": 2, "lim_hi": 3, "ramp_up": 4,
            "ramp_dn": 5, "logic": 6, "vw": 7, "min_up": 8, "min_dn": 9,
            "define_p": 10, "segment": 11, "segment_sum": 12, "cost_def": 13}
    inf = np.inf
    for t in range(T):
        # balance: sum_g p + sum_b d^pen = D_t
        ptr_parts.append(np.array([G + B], np.int64))
        col_parts.append(np.concatenate([col_index(G, t, P, g), pen_col_index(G, H, T, B, t, bus)]))
        val_parts.append(np.ones(G + B))
        lo_parts.append(np.array([dem[t]]))
        hi_parts.append(np.array([dem[t]]))
        row_kind_parts.append(np.array([KIND["balance"]], np.int8))
        row_sec_parts.append(np.array([-1], np.int32))
        if S:
            # sum_b delta_lb (sum_{g at b} p_g + d^pen_b) within D-dependent mid +- F
            ptr_parts.append(np.diff(sec.indptr).astype(np.int64))
            col_parts.append(np.where(sec_is_gen, col_index(G, t, P, np.minimum(sec.indices, G - 1)),
                                      pen_col_index(G, H, T, B, t, sec.indices - G)))
            val_parts.append(sec.data.copy())
            mid = data.sec_const * data.demand[t] / eta_p
            lo_parts.append(mid - F)
            hi_parts.append(mid + F)
            row_kind_parts.append(np.full(S, KIND["security"], np.int8))
            row_sec_parts.append(np.arange(S, dtype=np.int32))
        r_list, c_list, v_list, lo, hi, kind = [], [], [], [], [], []
        nrow = 0

        def add(rows_local, cols, vals):
            r_list.append(rows_local)
            c_list.append(cols)
            v_list.append(vals)

        def pp(tt, slot):
            return full_col_index(G, H, tt, slot, g, T)

        # p - p' - P^L u = 0
        rr = nrow + g
        add(rr, col_index(G, t, P, g), np.ones(G))
        add(rr, pp(t, 0), -np.ones(G))
        add(rr, col_index(G, t, U, g), -pmin)
        lo.append(np.zeros(G)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["define_p"]))
        nrow += G
        # p' - (P^U - P^L) u <= 0
        rr = nrow + g
        add(rr, pp(t, 0), np.ones(G))
        add(rr, col_index(G, t, U, g), -(pmax - pmin))
        lo.append(np.full(G, -inf)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["lim_hi"]))
        nrow += G
        if t >= 1:
            # (p'_t + P^L u_t) - (p'_{t-1} + P^L u_{t-1}) - RU u_{t-1} - SU v_t <= 0
            rr = nrow + g
            add(rr, pp(t, 0), np.ones(G))
            add(rr, col_index(G, t, U, g), pmin)
            add(rr, pp(t - 1, 0), -np.ones(G))
            add(rr, col_index(G, t - 1, U, g), -(pmin + ru))
            add(rr, col_index(G, t, V, g), -su)
            lo.append(np.full(G, -inf)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["ramp_up"]))
            nrow += G
            # (p'_{t-1} + P^L u_{t-1}) - (p'_t + P^L u_t) - RD u_t - SD w_t <= 0
            rr = nrow + g
            add(rr, pp(t - 1, 0), np.ones(G))
            add(rr, col_index(G, t - 1, U, g), pmin)
            add(rr, pp(t, 0), -np.ones(G))
            add(rr, col_index(G, t, U, g), -(pmin + ru))
            add(rr, col_index(G, t, W, g), -su)
            lo.append(np.full(G, -inf)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["ramp_dn"]))
            nrow += G
        # p_h - (P^U_h - P^U_{h-1}) u <= 0
        for h in range(H):
            rr = nrow + g
            add(rr, pp(t, 1 + h), np.ones(G))
            add(rr, col_index(G, t, U, g), -wd[:, h])
            lo.append(np.full(G, -inf)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["segment"]))
            nrow += G
        # sum_h p_h - p' = 0
        rr = nrow + g
        add(rr, pp(t, 0), -np.ones(G))
        for h in range(H):
            add(rr, pp(t, 1 + h), np.ones(G))
        lo.append(np.zeros(G)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["segment_sum"]))
        nrow += G
        # sum_h C_h p_h - c = 0
        rr = nrow + g
        for h in range(H):
            add(rr, pp(t, 1 + h), cs[:, h])
        add(rr, pp(t, H + 1), -np.ones(G))
        lo.append(np.zeros(G)); hi.append(np.zeros(G)); kind.append(np.full(G, KIND["cost_def"]))
        nrow += G
        nrow = _status_rows(add, data, t, nrow, lo, hi, kind, KIND)

        bptr, bcol, bval = _csr_from_coo(nrow, np.concatenate(r_list), np.concatenate(c_list),
                                         np.concatenate(v_list))
        ptr_parts.append(np.diff(bptr))
        col_parts.append(bcol)
        val_parts.append(bval)
        lo_parts.append(np.concatenate(lo))
        hi_parts.append(np.concatenate(hi))
        row_kind_parts.append(np.concatenate(kind).astype(np.int8))
        row_sec_parts.append(np.full(nrow, -1, np.int32))
        row_hour_parts.append(np.full(1 + S + nrow, t, np.int16))

    lens = np.concatenate(ptr_parts)
    row_ptr = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    col_idx = np.concatenate(col_parts).astype(np.int32)
    val = np.concatenate(val_parts).astype(np.float64)

    tt = np.arange(T)[:, None]
    gg = g[None, :]
    col_lo = np.zeros(n)
    col_hi = np.ones(n)
    col_hi[col_index(G, tt, P, gg).ravel()] = np.tile(pmax, T)
    col_hi[full_col_index(G, H, tt, 0, gg, T).ravel()] = np.tile(pmax - pmin, T)
    for h in range(H):
        col_hi[full_col_index(G, H, tt, 1 + h, gg, T).ravel()] = np.tile(wd[:, h], T)
    col_hi[full_col_index(G, H, tt, H + 1, gg, T).ravel()] = np.tile((cs * wd).sum(1), T)
    col_hi[pen_col_index(G, H, T, B, tt, bus[None, :]).ravel()] = (dem[:, None] * data.bus_share[None, :]).ravel()
    c = np.zeros(n)
    c[full_col_index(G, H, tt, H + 1, gg, T).ravel()] = 1.0
    c[col_index(G, tt, U, gg).ravel()] = np.tile(noload / eta_c, T)
    c[col_index(G, tt, V, gg).ravel()] = np.tile(data.startup_cost / eta_c, T)
    c[pen_col_index(G, H, T, B, tt, bus[None, :]).ravel()] = pen_cost * eta_p / eta_c

    meta = dict(config=cfg, G=G, T=T, eta_p=eta_p, eta_c=eta_c, formulation="full", segments=H,
                n_bus=B, pen_cost=pen_cost,
                row_kind=np.concatenate(row_kind_parts), row_kinds=KIND,
                row_hour=np.concatenate(row_hour_parts), row_sec=np.concatenate(row_sec_parts))
    return LP(len(lens), n, row_ptr, col_idx, val, np.concatenate(lo_parts), np.concatenate(hi_parts),
              col_lo, col_hi, c, 0.0, meta)


def feasible_point_full(data: SCUCData, lp: LP) -> np.ndarray:
    """The all-units-on dispatch of feasible_point in the full formulation's variables:
    segments filled cheapest first, no unserved demand."""
    G, T, H = data.cfg.n_gen, data.cfg.T, lp.meta["segments"]
    eta_p, eta_c = lp.meta["eta_p"], lp.meta["eta_c"]
    width, seg_cost, _ = segment_data(data, H)
    wd, cs = width / eta_p, seg_cost * eta_p / eta_c
    x = np.zeros(lp.n)
    g = np.arange(G)
    for t in range(T):
        p = data.demand[t] * data.p_max / data.p_max.sum() / eta_p
        x[col_index(G, t, U, g)] = 1.0
        x[col_index(G, t, P, g)] = p
        above = p - data.p_min / eta_p
        x[full_col_index(G, H, t, 0, g, T)] = above
        left = above.copy()
        cost = np.zeros(G)
        for h in range(H):
            s_h = np.clip(left, 0.0, wd[:, h])
            x[full_col_index(G, H, t, 1 + h, g, T)] = s_h
            cost += cs[:, h] * s_h
            left -= s_h
        x[full_col_index(G, H, t, H + 1, g, T)] = cost
    return x


def feasible_point(data: SCUCData, lp: LP) -> np.ndarray:
    """The all-units-on dispatch the line limits are built from (feasible by construction)."""
    G, T = data.cfg.n_gen, data.cfg.T
    x = np.zeros(lp.n)
    g = np.arange(G)
    for t in range(T):
        x[col_index(G, t, U, g)] = 1.0
        x[col_index(G, t, P, g)] = data.demand[t] * data.p_max / data.p_max.sum() / lp.meta["eta_p"]
    return x


def make_instance(cfg: SCUCConfig | str, seed: int, instance_scaling: bool = True,
                  formulation: str = "compact", segments: int = 3):
    """Generate (data, lp) for a preset name or config and a seed; `formulation` "compact"
    (u, v, w, p per generator-hour) or "full" (build_full_lp)."""
    if isinstance(cfg, str):
        cfg = PRESETS[cfg]
    if formulation == "full":
        data = make_scuc_data(cfg, seed, bus_rows=True)
        return data, build_full_lp(data, instance_scaling, segments)
    if formulation != "compact":
        raise ValueError(f"unknown formulation {formulation!r}")
    data = make_scuc_data(cfg, seed)
    return data, build_lp(data, instance_scaling)


# ----------------------------------------------------------------------------- small random LPs

def random_lp(rng: np.random.Generator, m: int, n: int, density: float = 0.6,
              box: float = 2.0, eq_frac: float = 0.2, range_frac: float = 0.3) -> LP:
    """A random bounded, feasible LP for exhaustive checks.

    A has N(0,1) entries at the given density (each row and column gets at least one
    entry). A hidden point x_f in the box fixes the row bounds so x_f is feasible:
    equality rows get lo = hi = a_i x_f, ranged rows an interval around it, the rest a
    one-sided bound (>= or <=). Column bounds are a finite box [-box, box] shifted at random.
    """
    mask = rng.random((m, n)) < density
    for i in range(m):
        if not mask[i].any():
            mask[i, rng.integers(n)] = True
    for j in range(n):
        if not mask[:, j].any():
            mask[rng.integers(m), j] = True
    Ad = np.where(mask, rng.standard_normal((m, n)), 0.0)
    col_lo = -box * rng.uniform(0.2, 1.0, n)
    col_hi = box * rng.uniform(0.2, 1.0, n)
    xf = rng.uniform(col_lo, col_hi)
    ax = Ad @ xf
    kind = rng.random(m)
    row_lo = np.full(m, -np.inf)
    row_hi = np.full(m, np.inf)
    for i in range(m):
        if kind[i] < eq_frac:
            row_lo[i] = row_hi[i] = ax[i]
        elif kind[i] < eq_frac + range_frac:
            row_lo[i] = ax[i] - rng.uniform(0.1, 1.0)
            row_hi[i] = ax[i] + rng.uniform(0.1, 1.0)
        elif kind[i] < eq_frac + range_frac + (1 - eq_frac - range_frac) / 2:
            row_lo[i] = ax[i] - rng.uniform(0.0, 0.5)
        else:
            row_hi[i] = ax[i] + rng.uniform(0.0, 0.5)
    c = rng.standard_normal(n)
    A = sp.csr_matrix(Ad)
    A.sort_indices()
    return LP(m, n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64),
              row_lo, row_hi, col_lo, col_hi, c, 0.0, {"x_feasible": xf})
