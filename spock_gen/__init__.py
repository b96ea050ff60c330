"""Seeded synthetic instances of the multistage risk-averse optimal control problem.

This module only draws inputs: tree shapes, node probabilities, dynamics, cost
weights, boxes, risk parameters and initial states. It contains none of the
solver's arithmetic and is the only code shared by the CPU oracle and the GPU
path.

Problem statement followed (paper section 4, "Multistage nested risk-averse
OCPs"): a scenario tree whose nodes are numbered breadth-first with contiguous
children (Fig. 1), node probabilities pi^i summing to one per stage, per-child
dynamics x^{i+} = A^{i+} x^i + B^{i+} u^i, quadratic stage costs
x'Q^{i+}x + u'R^{i+}u and terminal costs x'Q_N x, box constraints on states
and inputs, and an AV@R_a risk measure per nonleaf node (section 4.2).
Q, R and Q_N are diagonal in every workload here; they are stored as vectors.

Arrays (all float64 unless stated, row 0 of per-child data unused):
  anc   int32 [nn]        ancestor, anc[0] = -1
  prob        [nn]        node probability pi^i
  A           [nn,nx,nx]  dynamics of the edge anc(i) -> i (row-major)
  B           [nn,nx,nu]
  q           [nn,nx]     diag(Q^i), stage cost charged at child i
  r           [nn,nu]     diag(R^i)
  qN          [nn,nx]     diag(Q_N^j), read at leaves only
  xmin, xmax  [nn,nx]     state box at every node
  umin, umax  [nn,nu]     input box, read at nonleaf nodes only
  a_risk      [nn]        AV@R parameter a in [0,1], read at nonleaf nodes
  x0          [nx]        initial state
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

__all__ = [
    "Instance",
    "branching_anc",
    "rotation_scaled",
    "spectral_scaled",
    "make_config",
    "make_batch",
    "make_datacentre",
    "make_random_small",
    "CONFIG_NAMES",
    "dense_costs",
    "rotate_states_inputs",
]


@dataclass
class Instance:
    anc: np.ndarray
    prob: np.ndarray
    nx: int
    nu: int
    A: np.ndarray
    B: np.ndarray
    q: np.ndarray
    r: np.ndarray
    qN: np.ndarray
    xmin: np.ndarray
    xmax: np.ndarray
    umin: np.ndarray
    umax: np.ndarray
    a_risk: np.ndarray
    x0: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)
    # general conic risk (RiskData) and polyhedral constraints
    # (ConstraintData); None: AV@R_a per node and the boxes
    risk: object = None
    cons: object = None
    # dense cost matrices [num_nodes][nx][nx], [num_nodes][nu][nu] and
    # [num_nodes][nx][nx] (section 4.1); None: the diagonals q, r, qN
    Qm: object = None
    Rm: object = None
    QNm: object = None

    @property
    def num_nodes(self) -> int:
        return int(self.anc.shape[0])

    def copy(self) -> "Instance":
        return Instance(**{k: (v.copy() if isinstance(v, np.ndarray) else v)
                           for k, v in self.__dict__.items()})


def branching_anc(branching: Sequence[int]) -> np.ndarray:
    """Breadth-first ancestor array of a tree in which every node of stage t
    has branching[t] children (len(branching) = horizon N)."""
    anc = [-1]
    stage_nodes = [0]
    for b in branching:
        nxt = []
        for i in stage_nodes:
            for _ in range(int(b)):
                anc.append(i)
                nxt.append(len(anc) - 1)
        stage_nodes = nxt
    return np.asarray(anc, dtype=np.int32)


def _children_counts(anc: np.ndarray) -> np.ndarray:
    cnt = np.zeros(anc.shape[0], dtype=np.int64)
    for i in range(1, anc.shape[0]):
        cnt[anc[i]] += 1
    return cnt


def node_probabilities(anc: np.ndarray, cond: np.ndarray) -> np.ndarray:
    """pi^i from conditional probabilities cond[i] = pi^i / pi^{anc(i)}."""
    prob = np.zeros(anc.shape[0])
    prob[0] = 1.0
    for i in range(1, anc.shape[0]):
        prob[i] = prob[anc[i]] * cond[i]
    return prob


def rotation_scaled(rng: np.random.Generator, n: int, radius: float) -> np.ndarray:
    """radius * (Haar-orthogonal matrix); a planar rotation when n == 2."""
    if n == 1:
        return np.array([[radius * (1.0 if rng.random() < 0.5 else -1.0)]])
    if n == 2:
        th = rng.uniform(0.0, 2.0 * np.pi)
        c, s = np.cos(th), np.sin(th)
        return radius * np.array([[c, -s], [s, c]])
    g = rng.standard_normal((n, n))
    qm, rm = np.linalg.qr(g)
    qm = qm * np.sign(np.diag(rm))[None, :]
    return radius * qm


def spectral_scaled(rng: np.random.Generator, n: int, radius: float) -> np.ndarray:
    """radius * G / rho(G), G with i.i.d. N(0,1) entries."""
    g = rng.standard_normal((n, n))
    rho = np.max(np.abs(np.linalg.eigvals(g)))
    return radius * g / rho


def _cond_probs(rng, anc, kind, fixed=None):
    nn = anc.shape[0]
    cnt = _children_counts(anc)
    cond = np.ones(nn)
    first = {}
    for i in range(1, nn):
        first.setdefault(int(anc[i]), i)
    for par, fc in sorted(first.items()):
        n = int(cnt[par])
        if n == 1:
            cond[fc] = 1.0
            continue
        if kind == "uniform":
            w = np.full(n, 1.0 / n)
        elif kind == "dirichlet":
            w = rng.dirichlet(np.ones(n))
            w = np.maximum(w, 1e-3)
            w = w / w.sum()
        elif kind == "fixed":
            w = np.asarray(fixed, float)
            assert w.shape[0] == n
        else:
            raise ValueError(kind)
        cond[fc:fc + n] = w
    return cond


def _assemble(rng, anc, nx, nu, *, A_kind, A_radius, B_std, q_kind, r_val,
              qN_val, xbox, ubox, a_kind, prob_kind, x0_kind, name,
              prob_fixed=None):
    nn = anc.shape[0]
    cond = _cond_probs(rng, anc, prob_kind, prob_fixed)
    prob = node_probabilities(anc, cond)
    A = np.zeros((nn, nx, nx))
    B = np.zeros((nn, nx, nu))
    q = np.ones((nn, nx))
    r = np.full((nn, nu), r_val)
    for i in range(1, nn):
        rad = rng.uniform(*A_radius)
        A[i] = (rotation_scaled if A_kind == "rotation" else spectral_scaled)(rng, nx, rad)
        B[i] = B_std * rng.standard_normal((nx, nu))
        if q_kind == "diagU":
            q[i] = rng.uniform(0.5, 2.0, size=nx)
    qN = np.full((nn, nx), qN_val)
    xmin = np.full((nn, nx), -xbox)
    xmax = np.full((nn, nx), xbox)
    umin = np.full((nn, nu), -ubox)
    umax = np.full((nn, nu), ubox)
    cnt = _children_counts(anc)
    a_risk = np.zeros(nn)
    for i in range(nn):
        if cnt[i] > 0:
            a_risk[i] = a_kind(rng) if callable(a_kind) else float(a_kind)
    if x0_kind == "U2":
        x0 = rng.uniform(-2.0, 2.0, size=nx)
    else:
        x0 = rng.standard_normal(nx)
    return Instance(anc=anc, prob=prob, nx=nx, nu=nu, A=A, B=B, q=q, r=r, qN=qN,
                    xmin=xmin, xmax=xmax, umin=umin, umax=umax, a_risk=a_risk,
                    x0=x0, name=name)


CONFIG_NAMES = {
    1: "plain-fp64 nx2 nu1 N3 binary (15 nodes)",
    2: "single nx20 nu10 N10 b2x5 (223 nodes)",
    3: "large nx50 nu20 N15 b3x7 (20776 nodes)",
    4: "batched 512 uneven nx10 nu5",
    5: "diff 64 shared-tree nx20 nu10 N8 b2x4 (95 nodes)",
}


def make_config(k: int, seed: int = 0) -> Instance:
    """Single-instance workloads:

    1: 15-node tree, branching 2 for 3 stages, n_x 2, n_u 1;
    2: 223-node tree, branching 2 for 5 stages then 1 (N 10), n_x 20, n_u 10;
    3: 20 776-node tree, branching 3 for 7 stages then 1 (N 15, 2187
       scenarios), n_x 50, n_u 20;
    5: the 95-node tree shared by the 64-instance batch (branching 2 for 4
       stages then 1, N 8), n_x 20, n_u 10.
    """
    rng = np.random.default_rng(seed)
    if k == 1:
        anc = branching_anc([2, 2, 2])
        return _assemble(rng, anc, 2, 1, A_kind="rotation", A_radius=(0.9, 1.1),
                         B_std=1.0, q_kind="I", r_val=0.1, qN_val=1.0, xbox=5.0,
                         ubox=1.0, a_kind=0.5, prob_kind="uniform", x0_kind="U2",
                         name="config1")
    if k == 2:
        anc = branching_anc([2] * 5 + [1] * 5)
        return _assemble(rng, anc, 20, 10, A_kind="spectral", A_radius=(0.95, 1.05),
                         B_std=1.0 / np.sqrt(10.0), q_kind="diagU", r_val=0.1,
                         qN_val=1.0, xbox=10.0, ubox=2.0,
                         a_kind=lambda g: g.uniform(0.1, 0.9), prob_kind="dirichlet",
                         x0_kind="N", name="config2")
    if k == 3:
        anc = branching_anc([3] * 7 + [1] * 8)
        return _assemble(rng, anc, 50, 20, A_kind="rotation", A_radius=(0.9, 1.1),
                         B_std=1.0, q_kind="I", r_val=0.1, qN_val=1.0, xbox=5.0,
                         ubox=1.0, a_kind=0.2, prob_kind="dirichlet", x0_kind="U2",
                         name="config3")
    if k == 5:
        anc = branching_anc([2] * 4 + [1] * 4)
        return _assemble(rng, anc, 20, 10, A_kind="rotation", A_radius=(0.9, 1.1),
                         B_std=1.0, q_kind="I", r_val=0.1, qN_val=1.0, xbox=5.0,
                         ubox=1.0, a_kind=0.3, prob_kind="uniform", x0_kind="N",
                         name="config5")
    raise ValueError(f"no single-instance config {k}")


def make_batch(k: int, seed: int = 0, count: int | None = None) -> List[Instance]:
    """Batched workloads: 4 (512 uneven trees) and 5 (64 instances sharing one
    tree and its data, differing in x0)."""
    if k == 4:
        count = 512 if count is None else count
        out = []
        for b in range(count):
            rng = np.random.default_rng([seed, b])
            N = int(rng.integers(5, 13))
            kb = min(int(rng.integers(2, 7)), N)
            anc = branching_anc([2] * kb + [1] * (N - kb))
            inst = _assemble(rng, anc, 10, 5, A_kind="rotation", A_radius=(0.9, 1.1),
                             B_std=1.0, q_kind="I", r_val=0.1, qN_val=1.0, xbox=5.0,
                             ubox=1.0, a_kind=lambda g: g.uniform(0.1, 0.9),
                             prob_kind="uniform", x0_kind="N", name=f"config4[{b}]")
            inst.meta.update(N=N, k=kb)
            out.append(inst)
        return out
    if k == 5:
        count = 64 if count is None else count
        base = make_config(5, seed)
        out = []
        for b in range(count):
            rng = np.random.default_rng([seed, 1000 + b])
            inst = base.copy()
            inst.x0 = rng.standard_normal(base.nx)
            inst.name = f"config5[{b}]"
            out.append(inst)
        return out
    raise ValueError(f"no batched config {k}")


def make_datacentre(N: int, nx: int, d: int = 2, probs=(0.3, 0.7), a: float = 0.95,
                    x0_scale: float = 0.1) -> Instance:
    """The paper's data-centre thermal example (section 6, eq. dynamics-example):
    tridiagonal A(w) with diagonal 1 + (w-1)/d * (1 + (j-1)/nx) and off-diagonals
    0.01, B = I, Q = Q_N = I, R = 10 I, |x| <= 1, |u| <= 1.5, AV@R_a at every
    nonleaf node, binary tree with conditional probabilities (0.3, 0.7)."""
    anc = branching_anc([d] * N)
    nn = anc.shape[0]
    nu = nx
    cnt = _children_counts(anc)
    cond = np.ones(nn)
    first = {}
    for i in range(1, nn):
        first.setdefault(int(anc[i]), i)
    for par, fc in first.items():
        cond[fc:fc + d] = probs
    prob = node_probabilities(anc, cond)
    A = np.zeros((nn, nx, nx))
    B = np.zeros((nn, nx, nu))
    for i in range(1, nn):
        w = (i - first[int(anc[i])]) + 1  # disturbance value 1..d
        for j in range(1, nx + 1):
            A[i, j - 1, j - 1] = 1.0 + (w - 1) / d * (1.0 + (j - 1) / nx)
            if j >= 2:
                A[i, j - 1, j - 2] = 0.01
                A[i, j - 2, j - 1] = 0.01
        B[i] = np.eye(nx)
    a_risk = np.where(cnt > 0, a, 0.0)
    return Instance(anc=anc, prob=prob, nx=nx, nu=nu, A=A, B=B,
                    q=np.ones((nn, nx)), r=np.full((nn, nu), 10.0),
                    qN=np.ones((nn, nx)), xmin=-np.ones((nn, nx)),
                    xmax=np.ones((nn, nx)), umin=np.full((nn, nu), -1.5),
                    umax=np.full((nn, nu), 1.5), a_risk=a_risk,
                    x0=np.full(nx, x0_scale), name=f"datacentre N{N} nx{nx}")


def make_random_small(seed: int, branching: Sequence[int], nx: int, nu: int,
                      a: float | None = None, box: float = 5.0, ubox: float = 1.0,
                      q_kind: str = "diagU", prob_kind: str = "dirichlet") -> Instance:
    """Small random instance for tests (any branching pattern)."""
    rng = np.random.default_rng(seed)
    anc = branching_anc(branching)
    inst = _assemble(rng, anc, nx, nu, A_kind="rotation", A_radius=(0.9, 1.1),
                     B_std=1.0, q_kind=q_kind, r_val=0.1, qN_val=1.0, xbox=box,
                     ubox=ubox, a_kind=(lambda g: g.uniform(0.1, 0.9)) if a is None else a,
                     prob_kind=prob_kind, x0_kind="N", name=f"random{seed}")
    inst.r = rng.uniform(0.1, 1.0, size=inst.r.shape)
    inst.qN = rng.uniform(0.5, 2.0, size=inst.qN.shape)
    return inst


# ---------------------------------------------------------------- general conic risk and constraints
@dataclass
class RiskData:
    """Conic risk of every nonleaf node (section 4.3): E[i] [ny, n_i], F[i]
    [ny, nnu], b[i] [ny], kpos[i] leading rows of K in the nonnegative
    orthant (the rest in {0}); None at leaves."""
    E: list
    F: list
    b: list
    kpos: np.ndarray


@dataclass
class ConstraintData:
    """Polyhedral constraints Gamma_x x + Gamma_u u in [cmin, cmax] at
    nonleaf nodes and Gamma_N x in [cNmin, cNmax] at leaves (section 4.1)."""
    Gx: np.ndarray     # [nn, nc, nx]
    Gu: np.ndarray     # [nn, nc, nu]
    cmin: np.ndarray   # [nn, nc]
    cmax: np.ndarray
    GN: np.ndarray     # [nn, ncN, nx]
    cNmin: np.ndarray  # [nn, ncN]
    cNmax: np.ndarray


def _children_lists(anc):
    nn = len(anc)
    ch = [[] for _ in range(nn)]
    for i in range(1, nn):
        ch[int(anc[i])].append(i)
    return ch


def avar_as_conic(inst: Instance) -> RiskData:
    """AV@R_a of every nonleaf node written as a general conic risk:
    E = [a I; -I; 1'], F empty, b = (p, 0, 1), K = R^{2n}_+ x {0}."""
    ch = _children_lists(inst.anc)
    E, F, b = [None] * inst.num_nodes, [None] * inst.num_nodes, [None] * inst.num_nodes
    kpos = np.zeros(inst.num_nodes, dtype=np.int64)
    for i, c in enumerate(ch):
        if not c:
            continue
        n = len(c)
        p = inst.prob[c] / inst.prob[i]
        E[i] = np.vstack([inst.a_risk[i] * np.eye(n), -np.eye(n), np.ones((1, n))])
        F[i] = np.zeros((2 * n + 1, 0))
        b[i] = np.concatenate([p, np.zeros(n), [1.0]])
        kpos[i] = 2 * n
    return RiskData(E, F, b, kpos)


def mixture_risk(inst: Instance, kappa: float) -> RiskData:
    """rho(Z) = (1 - kappa) E^p[Z] + kappa max Z, the ambiguity set
    {mu = (1 - kappa) p + kappa nu, nu >= 0, 1'nu = 1} in the conic form
    E mu + F nu <=_K b with nu != 0: rows -nu <= 0 (nonnegative cone),
    mu - kappa nu = (1 - kappa) p and 1'nu = 1 (zero cone)."""
    ch = _children_lists(inst.anc)
    E, F, b = [None] * inst.num_nodes, [None] * inst.num_nodes, [None] * inst.num_nodes
    kpos = np.zeros(inst.num_nodes, dtype=np.int64)
    for i, c in enumerate(ch):
        if not c:
            continue
        n = len(c)
        p = inst.prob[c] / inst.prob[i]
        E[i] = np.vstack([np.zeros((n, n)), np.eye(n), np.zeros((1, n))])
        F[i] = np.vstack([-np.eye(n), -kappa * np.eye(n), np.ones((1, n))])
        b[i] = np.concatenate([np.zeros(n), (1.0 - kappa) * p, [1.0]])
        kpos[i] = n
    return RiskData(E, F, b, kpos)


def boxes_as_constraints(inst: Instance) -> ConstraintData:
    """The state/input boxes written as polyhedral constraints (Gamma = I)."""
    nn, nx, nu = inst.num_nodes, inst.nx, inst.nu
    Gx = np.zeros((nn, nx + nu, nx))
    Gu = np.zeros((nn, nx + nu, nu))
    Gx[:, :nx, :] = np.eye(nx)
    Gu[:, nx:, :] = np.eye(nu)
    return ConstraintData(Gx, Gu, np.concatenate([inst.xmin, inst.umin], axis=1),
                          np.concatenate([inst.xmax, inst.umax], axis=1),
                          np.tile(np.eye(nx), (nn, 1, 1)), inst.xmin.copy(), inst.xmax.copy())


def random_constraints(rng: np.random.Generator, inst: Instance, nc: int, ncN: int, bound: float) -> ConstraintData:
    """|Gamma_x x + Gamma_u u| <= bound row-wise (rows with unit norm, random
    directions) at nonleaf nodes and |Gamma_N x| <= bound at leaves."""
    nn, nx, nu = inst.num_nodes, inst.nx, inst.nu
    G = rng.standard_normal((nn, nc, nx + nu))
    G /= np.linalg.norm(G, axis=2, keepdims=True)
    GN = rng.standard_normal((nn, ncN, nx))
    GN /= np.linalg.norm(GN, axis=2, keepdims=True)
    return ConstraintData(G[:, :, :nx].copy(), G[:, :, nx:].copy(), np.full((nn, nc), -bound),
                          np.full((nn, nc), bound), GN, np.full((nn, ncN), -bound), np.full((nn, ncN), bound))


def make_general_small(seed: int, branching: Sequence[int], nx: int, nu: int, kappa: float = 0.4,
                       nc: int | None = None, ncN: int | None = None, bound: float = 2.0,
                       x0_scale: float = 0.5) -> Instance:
    """Small instance with the mixture risk (a conic risk with nu != 0) and
    random polyhedral constraints (nc rows at nonleaf nodes, ncN at leaves;
    None keeps the boxes)."""
    inst = make_random_small(seed, branching, nx, nu)
    rng = np.random.default_rng([seed, 77])
    inst.x0 = x0_scale * inst.x0 / max(1.0, np.max(np.abs(inst.x0)))
    inst.risk = mixture_risk(inst, kappa)
    if nc is not None:
        inst.cons = random_constraints(rng, inst, nc, ncN if ncN is not None else nx, bound)
    inst.name = f"general{seed}"
    return inst


def _random_spd(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    """U diag(lam) U' with U Haar-orthogonal and lam ~ U[lo, hi]."""
    g = rng.standard_normal((n, n))
    qm, rr = np.linalg.qr(g)
    qm = qm * np.sign(np.diag(rr))
    return (qm * rng.uniform(lo, hi, size=n)) @ qm.T


def dense_costs(inst: Instance, seed: int) -> Instance:
    """A copy of inst with dense symmetric positive definite Q^c, R^c, Q_N^j
    (eigenvalues in [0.5, 2], [0.1, 1], [0.5, 2]) in place of the diagonals."""
    out = inst.copy()
    rng = np.random.default_rng([seed, 91])
    nn, nx, nu = inst.num_nodes, inst.nx, inst.nu
    out.Qm = np.stack([_random_spd(rng, nx, 0.5, 2.0) for _ in range(nn)])
    out.Rm = np.stack([_random_spd(rng, nu, 0.1, 1.0) for _ in range(nn)])
    out.QNm = np.stack([_random_spd(rng, nx, 0.5, 2.0) for _ in range(nn)])
    out.name = inst.name + "+dense"
    return out


def rotate_states_inputs(inst: Instance, U: np.ndarray, W: np.ndarray) -> Instance:
    """The same problem in the coordinates x' = U x, u' = W u (U, W
    orthogonal): A' = U A U', B' = U B W', Q' = U Q U', R' = W R W',
    Q_N' = U Q_N U' (dense), x0' = U x0. The boxes are not invariant under
    the rotation and are widened to +-1e6 (callers keep them inactive)."""
    out = inst.copy()
    nn = inst.num_nodes
    out.A = np.stack([U @ inst.A[c] @ U.T for c in range(nn)])
    out.B = np.stack([U @ inst.B[c] @ W.T for c in range(nn)])
    Q = inst.Qm if inst.Qm is not None else np.stack([np.diag(q) for q in inst.q])
    R = inst.Rm if inst.Rm is not None else np.stack([np.diag(r) for r in inst.r])
    QN = inst.QNm if inst.QNm is not None else np.stack([np.diag(q) for q in inst.qN])
    out.Qm = np.stack([U @ Q[c] @ U.T for c in range(nn)])
    out.Rm = np.stack([W @ R[c] @ W.T for c in range(nn)])
    out.QNm = np.stack([U @ QN[c] @ U.T for c in range(nn)])
    out.x0 = U @ inst.x0
    big = 1e6
    out.xmin = np.full_like(inst.xmin, -big)
    out.xmax = np.full_like(inst.xmax, big)
    out.umin = np.full_like(inst.umin, -big)
    out.umax = np.full_like(inst.umax, big)
    out.name = inst.name + "+rotated"
    return out

