"""SUPG/PSPG-stabilised incompressible Navier-Stokes residual and Jacobian
(oracle; test infrastructure only), Sec. 5.

Equal-order Q_k/Q_k elements, BDF2 in time with constant step dt and history
u^n = u^{n-1} = u0, so the discrete time derivative is alpha (u - u0) with
alpha = 3 / (2 dt).  Force f = 0.

Residual (test functions v, q), eq. (ns) plus the SUPG and PSPG terms of
Sec. 5:
  F = (alpha (u - u0), v) + (u . grad u, v) + (nu grad u, grad v)
      - (p, div v) + (div u, q)
      + sum_K delta_1 (R(u, p), u . grad v)_K + sum_K delta_1 (R(u, p), grad q)_K
  R(u, p) = alpha (u - u0) + u . grad u + grad p - nu Lap u.

Readings where the paper is silent:
* delta_1 per quadrature point of the linearisation point u0 (Tezduyar type):
  delta_1 = [(2/dt)^2 + (2 |u0| / h_K)^2 + 9 (4 nu / h_K^2)^2]^(-1/2) with
  h_K = |K|^(1/d) / k; delta_1 is frozen (not differentiated).
* Lap u at a quadrature point is J^{-T} H J^{-1} of the reference Hessian H,
  exact on affine cells (the second derivatives of the cell map are
  neglected).
* Jacobian at (u0, p0 = 0): the Gateaux derivative of F with delta_1 frozen.
  Oseen variant: without the terms du . grad u0 and (R(u0), du . grad v).
* Velocity Dirichlet nodes on the whole boundary (identity rows), pressure
  unconstrained.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis
from .fem import Space, _assemble, constrain


def _qp_data(S: Space, cells=None):
    """Per cell and Gauss point: JxW, physical gradients and Laplacians of the
    Q_k basis, values; velocity and pressure use the same (equal-order) basis."""
    xq, J, det, invJ, JxW = S.geometry(cells)
    q1 = basis.gauss_rule(S.k + 1)[0]
    N, dN, H = basis.tensor_basis(S.dim, S.k, q1)
    G = np.einsum("qib,cqba->cqia", dN, invJ)  # [c, q, i, a]
    # Lap phi = sum_a sum_bc invJ[b,a] invJ[c,a] H[b,c]
    L = np.einsum("cqba,cqda,qibd->cqi", invJ, invJ, H)
    vol = JxW.sum(axis=1)
    return N, G, L, JxW, vol


def linearization_data(S: Space, u0: np.ndarray, nu: float, dt: float, cells=None):
    """u0, grad u0, R(u0, 0) and delta_1 at every Gauss point (of the given
    cells; all by default).  u0: blocked nodal velocity [dim*Nv]."""
    N, G, L, JxW, vol = _qp_data(S, cells)
    vdofs = S.vdofs if cells is None else S.vdofs[np.asarray(cells)]
    d = S.dim
    uq = np.zeros(JxW.shape + (d,))
    gu = np.zeros(JxW.shape + (d, d))  # [c, q, comp, a]
    lap = np.zeros(JxW.shape + (d,))
    for c in range(d):
        loc = u0[vdofs + c * S.Nv]  # [cells, nb]
        uq[..., c] = loc @ N.T
        gu[..., c, :] = np.einsum("ei,eqia->eqa", loc, G)
        lap[..., c] = np.einsum("ei,eqi->eq", loc, L)
    R0 = np.einsum("eqa,eqca->eqc", uq, gu) - nu * lap
    hK = vol ** (1.0 / d) / S.k
    speed = np.linalg.norm(uq, axis=-1)
    delta = ((2.0 / dt) ** 2 + (2.0 * speed / hK[:, None]) ** 2 + 9.0 * (4.0 * nu / hK[:, None] ** 2) ** 2) ** -0.5
    return {"u": uq, "grad": gu, "R0": R0, "delta": delta, "N": N, "G": G, "L": L, "JxW": JxW, "vdofs": vdofs}


def _local_fields(S, data, x):
    """Values, gradients and Laplacians of a blocked [u; p] vector at the qp."""
    N, G, L = data["N"], data["G"], data["L"]
    d = S.dim
    vdofs = data["vdofs"]
    ul = np.stack([x[vdofs + c * S.Nv] for c in range(d)], -1)  # [e, i, c]
    pl = x[d * S.Nv:][vdofs]  # equal order: same local numbering
    u = np.einsum("qi,eic->eqc", N, ul)
    gu = np.einsum("eqia,eic->eqca", G, ul)
    lu = np.einsum("eqi,eic->eqc", L, ul)
    p = pl @ N.T
    gp = np.einsum("eqia,ei->eqa", G, pl)
    return u, gu, lu, p, gp


def _assemble_test(S, val_u, grad_u, val_p, grad_p, data):
    """Integrate test-function coefficients: val_u [e,q,c] multiplies v_c,
    grad_u [e,q,c,a] multiplies d_a v_c, val_p multiplies q, grad_p [e,q,a]
    multiplies d_a q."""
    N, G, JxW = data["N"], data["G"], data["JxW"]
    vdofs = data["vdofs"]
    d = S.dim
    out = np.zeros(d * S.Nv + S.Nv)
    for c in range(d):
        loc = np.einsum("eq,qi->ei", JxW * val_u[..., c], N) + np.einsum("eq,eqa,eqia->ei", JxW, grad_u[..., c, :], G)
        np.add.at(out, (vdofs + c * S.Nv).ravel(), loc.ravel())
    loc = np.einsum("eq,qi->ei", JxW * val_p, N) + np.einsum("eq,eqa,eqia->ei", JxW, grad_p, G)
    np.add.at(out, (vdofs + d * S.Nv).ravel(), loc.ravel())
    return out


def residual(S: Space, x: np.ndarray, u0: np.ndarray, nu: float, dt: float, data=None):
    """F(u, p) tested with every basis function (no constraints), with delta_1
    frozen at the linearisation point u0."""
    if data is None:
        data = linearization_data(S, u0, nu, dt)
    alpha = 1.5 / dt
    d = S.dim
    u, gu, lu, p, gp = _local_fields(S, data, x)
    u0q = data["u"]
    dl = data["delta"][..., None]
    conv = np.einsum("eqa,eqca->eqc", u, gu)
    R = alpha * (u - u0q) + conv + gp - nu * lu
    val_u = alpha * (u - u0q) + conv
    grad_u = nu * gu - p[..., None, None] * np.eye(d)[None, None] + dl[..., None] * R[..., :, None] * u[..., None, :]
    val_p = np.einsum("eqcc->eq", gu)
    grad_p = dl * R
    return _assemble_test(S, val_u, grad_u, val_p, grad_p, data)


def jacobian_apply(S: Space, dx: np.ndarray, data, nu: float, dt: float, newton: bool = True):
    """J(u0, 0) dx tested with every basis function (no constraints)."""
    alpha = 1.5 / dt
    d = S.dim
    w, gw, lw, P, gP = _local_fields(S, data, dx)
    u0, U, R0 = data["u"], data["grad"], data["R0"]
    dl = data["delta"][..., None]
    conv = np.einsum("eqa,eqca->eqc", u0, gw)  # u0 . grad du
    newt = np.einsum("eqa,eqca->eqc", w, U) if newton else 0.0  # du . grad u0
    Rl = alpha * w + newt + conv + gP - nu * lw
    val_u = alpha * w + newt + conv
    grad_u = nu * gw - P[..., None, None] * np.eye(d)[None, None] + dl[..., None] * Rl[..., :, None] * u0[..., None, :]
    if newton:
        grad_u = grad_u + dl[..., None] * R0[..., :, None] * w[..., None, :]
    val_p = np.einsum("eqcc->eq", gw)
    grad_p = dl * Rl
    return _assemble_test(S, val_u, grad_u, val_p, grad_p, data)


def ns_dirichlet_mask(S: Space):
    m = np.zeros(S.dim * S.Nv + S.Nv, dtype=bool)
    for c in range(S.dim):
        m[c * S.Nv:(c + 1) * S.Nv] = S.dirichlet
    return m


def constrained_jacobian_apply(S, dx, data, nu, dt, newton=True):
    """Constrained Jacobian: identity on Dirichlet rows, Dirichlet source
    values ignored elsewhere."""
    mask = ns_dirichlet_mask(S)
    y = jacobian_apply(S, np.where(mask, 0.0, dx), data, nu, dt, newton)
    y[mask] = dx[mask]
    return y


def jacobian_matrix(S: Space, data, nu, dt, newton=True):
    """Assembled constrained Jacobian (CSR) by applying it to unit vectors
    cell by cell is too slow; assemble element matrices by full quadrature."""
    alpha = 1.5 / dt
    d = S.dim
    N, G, L, JxW = data["N"], data["G"], data["L"], data["JxW"]
    u0, U, R0 = data["u"], data["grad"], data["R0"]
    dl = data["delta"]
    nb = N.shape[1]
    ne = JxW.shape[0]
    # trial quantities per basis j: value N, grad G, lap L
    a_dot_grad = np.einsum("eqa,eqja->eqj", u0, G)  # u0 . grad phi_j
    nd = d + 1
    E = np.zeros((ne, nd, nb, nd, nb))
    W = JxW
    I = np.eye(d)
    for c in range(d):  # test component (velocity)
        for cp in range(d):  # trial component
            # Galerkin value part: alpha phi_j + (du . grad u0)_c + (u0 . grad du)_c
            rl = (alpha * N[None] * (c == cp) + a_dot_grad * (c == cp)
                  - nu * L * (c == cp))  # [e,q,j]  R_lin_c for du = phi_j e_cp, without newton
            val = alpha * N[None] * (c == cp) + a_dot_grad * (c == cp)
            if newton:
                val = val + N[None] * U[..., c, cp][..., None]
                rl = rl + N[None] * U[..., c, cp][..., None]
            # test: v = phi_i e_c -> value phi_i, grad d_a phi_i
            E[:, c, :, cp, :] += np.einsum("eq,qi,eqj->eij", W, N, val)
            E[:, c, :, cp, :] += (c == cp) * nu * np.einsum("eq,eqia,eqja->eij", W, G, G)
            # SUPG: delta (R_lin_c, u0 . grad phi_i)
            E[:, c, :, cp, :] += np.einsum("eq,eqi,eqj->eij", W * dl, a_dot_grad, rl)
            if newton:  # delta (R0_c, phi_j d_cp phi_i)
                E[:, c, :, cp, :] += np.einsum("eq,eqi,qj->eij", W * dl * R0[..., c], G[..., cp], N)
        # pressure trial: -(dp, d_c phi_i) + delta (d_c psi_j, u0 . grad phi_i)
        E[:, c, :, d, :] += -np.einsum("eq,eqi,qj->eij", W, G[..., c], N)
        E[:, c, :, d, :] += np.einsum("eq,eqi,eqj->eij", W * dl, a_dot_grad, G[..., c])
    for cp in range(d):  # pressure test, velocity trial
        rl_all = np.zeros((ne, JxW.shape[1], d, nb))
        for c in range(d):
            rl = alpha * N[None] * (c == cp) + a_dot_grad * (c == cp) - nu * L * (c == cp)
            if newton:
                rl = rl + N[None] * U[..., c, cp][..., None]
            rl_all[:, :, c, :] = rl
        E[:, d, :, cp, :] += np.einsum("eq,qi,eqj->eij", W, N, G[..., cp])  # (div du, q)
        E[:, d, :, cp, :] += np.einsum("eq,eqic,eqcj->eij", W * dl, G, rl_all)  # PSPG
    E[:, d, :, d, :] += np.einsum("eq,eqia,eqja->eij", W * dl, G, G)
    del I
    l2g = np.concatenate([data["vdofs"] + c * S.Nv for c in range(nd)], axis=1)
    K = _assemble(l2g, l2g, E.reshape(ne, nd * nb, nd * nb), (nd * S.Nv, nd * S.Nv))
    return constrain(K, ns_dirichlet_mask(S))


def sampled_jacobian_rows(S: Space, dx, u0, nu, dt, rows, newton=True):
    """Rows of the constrained Jacobian applied to dx, from the cells that
    contain them only (for meshes too large for a full evaluation)."""
    from .fem import cells_containing

    rows = np.asarray(rows)
    cells = cells_containing(S, rows)
    data = linearization_data(S, u0, nu, dt, cells)
    mask = ns_dirichlet_mask(S)
    y = jacobian_apply(S, np.where(mask, 0.0, dx), data, nu, dt, newton)
    y[mask] = dx[mask]
    return y[rows]
