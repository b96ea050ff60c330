"""The linear operator L, its adjoint L*, and ||L||.

L follows the definition of eta in section 5.2 (operator splitting); L* is
written out column by column from that definition; ||L|| uses the remark after
it: after a column permutation L is block diagonal, so ||L|| is the largest
spectral norm of its blocks.
"""
from __future__ import annotations

import numpy as np

from .layout import Layout


def L_apply(lay: Layout, inst, z: np.ndarray) -> np.ndarray:
    nx, nu = lay.nx, lay.nu
    eta = np.zeros(lay.n_eta)
    for i in lay.nonleaf:
        ny = lay.ny[i]
        y = z[lay.y_off[i]: lay.y_off[i] + ny]
        eta[lay.e1y[i]: lay.e1y[i] + ny] = y
        eta[lay.e1s[i]] = z[lay.s_off[i]] - lay.b_vector(i) @ y
        Gx, Gu, _, _ = lay.gamma(inst, i)
        eta[lay.e1c[i]: lay.e1c[i] + lay.nc] = (Gx @ z[lay.x_off[i]: lay.x_off[i] + nx]
                                                + Gu @ z[lay.u_off[i]: lay.u_off[i] + nu])
    for c in range(1, lay.num_nodes):
        i = lay.anc[c]
        xi, ui = z[lay.x_off[i]: lay.x_off[i] + nx], z[lay.u_off[i]: lay.u_off[i] + nu]
        if lay.dense_costs:
            Qh, Rh, _ = lay.cost_roots(inst, c)
            eta[lay.e2x[c]: lay.e2x[c] + nx] = Qh @ xi
            eta[lay.e2u[c]: lay.e2u[c] + nu] = Rh @ ui
        else:
            eta[lay.e2x[c]: lay.e2x[c] + nx] = np.sqrt(inst.q[c]) * xi
            eta[lay.e2u[c]: lay.e2u[c] + nu] = np.sqrt(inst.r[c]) * ui
        eta[lay.e2a[c]] = 0.5 * z[lay.tau_off[c]]
        eta[lay.e2b[c]] = 0.5 * z[lay.tau_off[c]]
    for j in lay.leaves:
        xj = z[lay.x_off[j]: lay.x_off[j] + nx]
        eta[lay.e3x[j]: lay.e3x[j] + lay.ncN] = lay.gamma_N(inst, j)[0] @ xj
        if lay.dense_costs:
            eta[lay.e3q[j]: lay.e3q[j] + nx] = lay.cost_roots(inst, j)[2] @ xj
        else:
            eta[lay.e3q[j]: lay.e3q[j] + nx] = np.sqrt(inst.qN[j]) * xj
        eta[lay.e3a[j]] = 0.5 * z[lay.s_off[j]]
        eta[lay.e3b[j]] = 0.5 * z[lay.s_off[j]]
    return eta


def Lt_apply(lay: Layout, inst, eta: np.ndarray) -> np.ndarray:
    nx, nu = lay.nx, lay.nu
    z = np.zeros(lay.n_z)
    for i in lay.nonleaf:
        ny = lay.ny[i]
        e_y = eta[lay.e1y[i]: lay.e1y[i] + ny]
        e_s = eta[lay.e1s[i]]
        z[lay.y_off[i]: lay.y_off[i] + ny] += e_y - lay.b_vector(i) * e_s
        z[lay.s_off[i]] += e_s
        Gx, Gu, _, _ = lay.gamma(inst, i)
        e_c = eta[lay.e1c[i]: lay.e1c[i] + lay.nc]
        z[lay.x_off[i]: lay.x_off[i] + nx] += Gx.T @ e_c
        z[lay.u_off[i]: lay.u_off[i] + nu] += Gu.T @ e_c
    for c in range(1, lay.num_nodes):
        i = lay.anc[c]
        ex, eu = eta[lay.e2x[c]: lay.e2x[c] + nx], eta[lay.e2u[c]: lay.e2u[c] + nu]
        if lay.dense_costs:
            Qh, Rh, _ = lay.cost_roots(inst, c)
            z[lay.x_off[i]: lay.x_off[i] + nx] += Qh.T @ ex
            z[lay.u_off[i]: lay.u_off[i] + nu] += Rh.T @ eu
        else:
            z[lay.x_off[i]: lay.x_off[i] + nx] += np.sqrt(inst.q[c]) * ex
            z[lay.u_off[i]: lay.u_off[i] + nu] += np.sqrt(inst.r[c]) * eu
        z[lay.tau_off[c]] += 0.5 * (eta[lay.e2a[c]] + eta[lay.e2b[c]])
    for j in lay.leaves:
        eq = eta[lay.e3q[j]: lay.e3q[j] + nx]
        qn = lay.cost_roots(inst, j)[2].T @ eq if lay.dense_costs else np.sqrt(inst.qN[j]) * eq
        z[lay.x_off[j]: lay.x_off[j] + nx] += lay.gamma_N(inst, j)[0].T @ eta[lay.e3x[j]: lay.e3x[j] + lay.ncN] + qn
        z[lay.s_off[j]] += 0.5 * (eta[lay.e3a[j]] + eta[lay.e3b[j]])
    return z


def dense_L(lay: Layout, inst) -> np.ndarray:
    """L as a dense matrix, column by column (small trees only)."""
    M = np.zeros((lay.n_eta, lay.n_z))
    e = np.zeros(lay.n_z)
    for k in range(lay.n_z):
        e[k] = 1.0
        M[:, k] = L_apply(lay, inst, e)
        e[k] = 0.0
    return M


def _block_columns(lay: Layout):
    """Column groups of the block-diagonal permutation of L: each group's
    columns touch rows that no other group touches."""
    nx, nu = lay.nx, lay.nu
    groups = []
    for i in lay.nonleaf:
        n = len(lay.children[i])
        groups.append(list(range(lay.x_off[i], lay.x_off[i] + nx))
                      + list(range(lay.u_off[i], lay.u_off[i] + nu)))
        groups.append(list(range(lay.y_off[i], lay.y_off[i] + lay.ny[i])) + [lay.s_off[i]])
        for c in lay.children[i]:
            groups.append([lay.tau_off[c]])
    for j in lay.leaves:
        groups.append(list(range(lay.x_off[j], lay.x_off[j] + nx)) + [lay.s_off[j]])
    return groups


def norm_L(lay: Layout, inst) -> float:
    """max over blocks of the largest singular value (numpy SVD).

    Column groups of different blocks reach disjoint rows, so applying L to
    the sum of the k-th column of every group yields the k-th column of every
    block at once; a second probe weighted by the group number tells which
    block each nonzero row belongs to."""
    groups = _block_columns(lay)
    width = max(len(g) for g in groups)
    cols, labels = [], []
    for k in range(width):
        probe = np.zeros(lay.n_z)
        tagged = np.zeros(lay.n_z)
        for gi, g in enumerate(groups):
            if k < len(g):
                probe[g[k]] = 1.0
                tagged[g[k]] = gi + 1.0
        col = L_apply(lay, inst, probe)
        tag = L_apply(lay, inst, tagged)
        lab = np.zeros(lay.n_eta, dtype=np.int64)
        nz = col != 0.0
        lab[nz] = np.rint(tag[nz] / col[nz]).astype(np.int64) - 1
        lab[~nz] = -1
        cols.append(col)
        labels.append(lab)
    row_group = np.full(lay.n_eta, -1, dtype=np.int64)
    for lab in labels:
        row_group = np.where(lab >= 0, lab, row_group)
    order = np.argsort(row_group, kind="stable")
    sorted_groups = row_group[order]
    best = 0.0
    starts = np.searchsorted(sorted_groups, np.arange(len(groups)), side="left")
    ends = np.searchsorted(sorted_groups, np.arange(len(groups)), side="right")
    for gi, g in enumerate(groups):
        rows = order[starts[gi]:ends[gi]]
        if rows.size == 0:
            continue
        Mb = np.stack([cols[k][rows] for k in range(len(g))], axis=1)
        s = np.linalg.svd(Mb, compute_uv=False)
        best = max(best, float(s[0]))
    return best
