"""Second, independent implementation of the oracle's CRK-SPH chain for tiny N.

Dense NumPy: every pair quantity is an (N, N) array, sums are einsum
contractions and the 3x3 solves go through numpy.linalg.  Written separately
from ``oracle/crk_oracle.cpp`` (different structure, different order of
operations) so that agreement at roundoff level pins the oracle's code.  Used
only by the oracle's pin tests.
"""

import numpy as np

C_W = 495.0 / (32.0 * np.pi)
C_F = -1155.0 / (4.0 * np.pi)


def separations(g):
    P = np.stack([g["x"], g["y"], g["z"]], axis=1)
    d = P[:, None, :] - P[None, :, :]
    d = d - np.floor(d + 0.5)  # minimum image into [-1/2, 1/2)
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    return d, r


def wendland(r, H):
    """W and F (grad_i W = F x_ij) for support H (broadcasting)."""
    q = r / H
    t = np.clip(1.0 - q, 0.0, None)
    W = C_W / H ** 3 * t ** 6 * (1.0 + 6.0 * q + 35.0 / 3.0 * q * q)
    F = C_F / H ** 5 * (1.0 + 5.0 * q) * t ** 5
    return W, F


def chain(g, corr_override=None):
    d, r = separations(g)
    n = r.shape[0]
    h = np.asarray(g["h"])
    Hi = (2.0 * h)[:, None]
    Hj = (2.0 * h)[None, :]
    Wi, Fi = wendland(r, Hi)  # W(r_ij, h_i)
    Wj, Fj = wendland(r, Hj)  # W(r_ij, h_j)
    S = Wi.sum(axis=1)  # includes the diagonal W(0, h_i)
    V = 1.0 / S
    rho = g["m"] * S
    # moments: sums over j weighted by V_j (the diagonal contributes W(0) terms)
    w = Wi * V[None, :]
    f = Fi * V[None, :]
    dW = f[:, :, None] * d  # V_j d_c W_ij
    m0 = w.sum(1)
    m1 = np.einsum("ij,ija->ia", w, d)
    m2 = np.einsum("ij,ija,ijb->iab", w, d, d)
    g0 = dW.sum(1)
    eye = np.eye(3)
    g1 = m0[:, None, None] * eye[None] + np.einsum("ija,ijc->iac", d, dW)
    g2 = (np.einsum("ac,ib->iabc", eye, m1) + np.einsum("bc,ia->iabc", eye, m1)
          + np.einsum("ija,ijb,ijc->iabc", d, d, dW))
    B = -np.linalg.solve(m2, m1[:, :, None])[:, :, 0]
    A = 1.0 / (m0 + np.einsum("ia,ia->i", B, m1))
    rhs = g1 + np.einsum("iabc,ib->iac", g2, B)  # rhs[i, a, c]
    dB = -np.linalg.solve(m2, rhs)  # dB[i, a, c] = d_c B^a
    dA = -(A ** 2)[:, None] * (g0 + np.einsum("ia,iac->ic", B, g1) + np.einsum("ia,iac->ic", m1, dB))
    if corr_override is not None:
        A, B, dA, dB = corr_override
    # corrected-kernel gradients G_ij (own kernel) and G_ji (neighbour's kernel)
    lin_i = 1.0 + np.einsum("ia,ija->ij", B, d)
    Gij = (dA[:, None, :] * (lin_i * Wi)[:, :, None]
           + A[:, None, None] * (np.einsum("iac,ija->ijc", dB, d) + B[:, None, :]) * Wi[:, :, None]
           + (A[:, None] * lin_i * Fi)[:, :, None] * d)
    # G_ji uses particle j's corrections and x_ji = -x_ij
    lin_j = 1.0 - np.einsum("ja,ija->ij", B, d)
    Gji = (dA[None, :, :] * (lin_j * Wj)[:, :, None]
           + A[None, :, None] * (-np.einsum("jac,ija->ijc", dB, d) + B[None, :, :]) * Wj[:, :, None]
           - (A[None, :] * lin_j * Fj)[:, :, None] * d)
    P = (g["gamma"] - 1.0) * rho * g["u"]
    Hmax = np.maximum(Hi, Hj)
    mask = (r < Hmax) & ~np.eye(n, dtype=bool)
    coef = -0.5 * V[:, None] * V[None, :] * (P[:, None] + P[None, :]) * mask
    Fij = coef[:, :, None] * (Gij - Gji)
    v = np.stack([g["vx"], g["vy"], g["vz"]], axis=1)
    vij = v[:, None, :] - v[None, :, :]
    a = Fij.sum(1) / g["m"][:, None]
    dudt = -0.5 * np.einsum("ijc,ijc->i", Fij, vij) / g["m"]
    return dict(V=V, rho=rho, m0=m0, m1=m1, m2=m2, g0=g0, g1=g1, g2=g2, A=A, B=B, dA=dA, dB=dB,
                a=a, dudt=dudt, d=d, r=r, Wi=Wi, Fi=Fi, Gij=Gij, Gji=Gji, Fij=Fij, vij=vij)


def extras_and_viscosity(g, dn, Cl=1.0, Cq=2.0, eps_q=0.01):
    """CRK density, gradients of v and u, and the forces with the artificial
    viscosity, densely from a chain() result (same readings as the oracle:
    gather support r < 2h_i for the extras; per force pair the van Leer limiter
    on s_k = x.(dv_k x), midpoint-reconstructed velocities, Q_k =
    rho_k (-Cl c_k mu_k + Cq mu_k^2) added to the pressures)."""
    d, r = dn["d"], dn["r"]
    n = r.shape[0]
    h = np.asarray(g["h"])
    off = ~np.eye(n, dtype=bool)
    gather = (r < (2.0 * h)[:, None]) & off
    WR = dn["A"][:, None] * (1.0 + np.einsum("ia,ija->ij", dn["B"], d)) * dn["Wi"]
    rhoR = (WR * g["m"][None, :]).sum(1)  # the diagonal carries the self term
    v = np.stack([g["vx"], g["vy"], g["vz"]], axis=1)
    wgt = dn["V"][None, :] * gather
    dv = np.einsum("ij,ija,ijc->iac", wgt, v[None, :, :] - v[:, None, :], dn["Gij"])
    du = np.einsum("ij,ij,ijc->ic", wgt, g["u"][None, :] - g["u"][:, None], dn["Gij"])
    # viscosity per ordered pair (i, j)
    Di = np.einsum("iac,ijc->ija", dv, d)
    Dj = np.einsum("jac,ijc->ija", dv, d)
    si = np.einsum("ija,ija->ij", d, Di)
    sj = np.einsum("ija,ija->ij", d, Dj)
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(si * sj > 0, 4.0 * si * sj / (si + sj) ** 2, 0.0)
    w = (v[:, None, :] - v[None, :, :]) - 0.5 * phi[:, :, None] * (Di + Dj)
    wx = np.einsum("ija,ija->ij", w, d)
    cs = np.sqrt(g["gamma"] * (g["gamma"] - 1.0) * g["u"])
    r2 = r * r

    def q(side_h, side_rho, side_c):
        mu = np.minimum(0.0, side_h * wx / (r2 + eps_q * side_h ** 2))
        return side_rho * (-Cl * side_c * mu + Cq * mu * mu)

    Q = q(h[:, None], dn["rho"][:, None], cs[:, None]) + q(h[None, :], dn["rho"][None, :], cs[None, :])
    # forces: rebuild the pair sums with P_i + P_j + Q_ij
    Hmax = np.maximum(2.0 * h[:, None], 2.0 * h[None, :])
    mask = (r < Hmax) & off
    P = (g["gamma"] - 1.0) * dn["rho"] * g["u"]
    V = dn["V"]
    coef = -0.5 * V[:, None] * V[None, :] * (P[:, None] + P[None, :] + Q) * mask
    Fij = coef[:, :, None] * (dn["Gij"] - dn["Gji"])
    vij = v[:, None, :] - v[None, :, :]
    a = Fij.sum(1) / g["m"][:, None]
    dudt = -0.5 * np.einsum("ijc,ijc->i", Fij, vij) / g["m"]
    return dict(rhoR=rhoR, dv=dv, du=du, a=a, dudt=dudt)
