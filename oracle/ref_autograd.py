"""Independent float64 reference of the summed Kalman chi2 and its map gradient.

TEST INFRASTRUCTURE ONLY.  A second implementation of the oracle's fit in
plain PyTorch (CPU, float64) used to pin gradients: the propagation Jacobian
comes from automatic differentiation of the helix step (not from the analytic
derivative the C oracle writes out), and the gradient of the chi2 sum with
respect to a per-(sector, row) correction map comes from reverse-mode
autograd through everything (start, Jacobian, gain, chi2).

Reading of the method (the paper gives none): three-point helix start at the
outermost hit, inward extended Kalman filter without process noise,
chi2 = sum of predicted-residual chi2 over the hits after the first.
"""
from __future__ import annotations

import numpy as np
import torch
from torch.func import jacrev, vmap

C_LIGHT = 0.00299792458


def _g(u):
    """asin(u)/u, continuous at 0 with a safe gradient."""
    small = u.abs() < 1e-2
    us = torch.where(small, torch.full_like(u, 0.5), u)
    u2 = u * u
    ser = 1.0 + u2 * (1.0 / 6.0 + u2 * (3.0 / 40.0 + u2 * (5.0 / 112.0)))
    return torch.where(small, ser, torch.asin(us) / us)


def helix_step(p, dx, bz):
    """Single state p[5] = (y, z, sin phi, tan lambda, q/pT) moved by dx along x."""
    y, z, s, t, w = p[0], p[1], p[2], p[3], p[4]
    kap = -C_LIGHT * bz * w
    s2 = s + kap * dx
    c1 = torch.sqrt(1.0 - s * s)
    c2 = torch.sqrt(1.0 - s2 * s2)
    T = (s + s2) / (c1 + c2)
    chord = torch.abs(dx) * torch.sqrt(1.0 + T * T)
    arc = torch.sign(dx) * chord * _g(kap * chord / 2.0)
    return torch.stack([y + dx * T, z + t * arc, s2, t, w])


def chi2_sum_torch(map_t: torch.Tensor, seeds: dict, y, z, row_x, *, bz, sigma_y, sigma_z,
                   var_sin0, var_tgl0, var_qpt0, include=None) -> torch.Tensor:
    """Sum of chi2 over the seeds (or the ``include`` mask of them)."""
    dt = torch.float64
    offs = np.asarray(seeds["offsets"])
    hits = np.asarray(seeds["hits"])
    sec = np.asarray(seeds["sector"])
    fr = np.asarray(seeds["first_row"])
    n = np.diff(offs)
    if include is not None:
        keep = np.nonzero(include)[0]
    else:
        keep = np.arange(len(n))
    T = len(keep)
    nmax = int(n[keep].max())
    K = np.zeros((T, nmax), np.int64)
    valid = np.zeros((T, nmax), bool)
    for j, i in enumerate(keep):
        K[j, :n[i]] = hits[offs[i]:offs[i + 1]]
        valid[j, :n[i]] = True
    rows = fr[keep][:, None] + np.arange(nmax)[None, :]
    rows = np.where(valid, rows, 0)
    secs = np.repeat(sec[keep][:, None], nmax, 1)
    yv = torch.as_tensor(np.asarray(y, np.float64)[K], dtype=dt)
    zv = torch.as_tensor(np.asarray(z, np.float64)[K], dtype=dt)
    xv = torch.as_tensor(np.asarray(row_x, np.float64)[rows], dtype=dt)
    ms = torch.as_tensor(secs)
    mr = torch.as_tensor(rows)
    ym = yv - map_t[ms, mr, 0]
    zm = zv - map_t[ms, mr, 1]
    nn = torch.as_tensor(n[keep])
    ar = torch.arange(T)
    a = nn - 1
    b = (nn - 1) // 2
    c = torch.zeros_like(nn)
    xa, ya, za = xv[ar, a], ym[ar, a], zm[ar, a]
    xb, yb = xv[ar, b], ym[ar, b]
    xc, yc, zc = xv[ar, c], ym[ar, c], zm[ar, c]
    bcx, bcy = xb - xc, yb - yc
    abx, aby = xa - xb, ya - yb
    acx, acy = xa - xc, ya - yc
    lbc = torch.sqrt(bcx ** 2 + bcy ** 2)
    lab = torch.sqrt(abx ** 2 + aby ** 2)
    lac = torch.sqrt(acx ** 2 + acy ** 2)
    kap0 = 2.0 * (bcx * aby - bcy * abx) / (lbc * lab * lac)
    phia = torch.atan2(aby, abx) + torch.asin(kap0 * lab / 2.0)
    s0 = torch.sin(phia)
    t0 = (za - zc) / (lac * _g(kap0 * lac / 2.0))
    w0 = -kap0 / (C_LIGHT * bz)
    p = torch.stack([ya, za, s0, t0, w0], dim=1)
    C = torch.diag(torch.tensor([sigma_y ** 2, sigma_z ** 2, var_sin0, var_tgl0, var_qpt0],
                                dtype=dt)).expand(T, 5, 5)
    V = torch.tensor([sigma_y ** 2, sigma_z ** 2], dtype=dt)
    chi2 = torch.zeros(T, dtype=dt)
    step = vmap(helix_step, in_dims=(0, 0, None))
    jac = vmap(jacrev(helix_step, argnums=0), in_dims=(0, 0, None))
    for j in range(1, nmax):
        k = nn - 1 - j
        act = k >= 0
        kk = torch.clamp(k, min=0)
        dx = xv[ar, kk] - xv[ar, torch.clamp(k + 1, max=nmax - 1)]
        dx = torch.where(act, dx, torch.ones_like(dx) * -1.0)
        pp = step(p, dx, bz)
        F = jac(p, dx, bz)
        Cp = F @ C @ F.transpose(1, 2)
        r = torch.stack([ym[ar, kk] - pp[:, 0], zm[ar, kk] - pp[:, 1]], dim=1)
        S = Cp[:, :2, :2] + torch.diag(V)
        Si = torch.linalg.inv(S)
        Kg = Cp[:, :, :2] @ Si
        pn = pp + (Kg @ r[:, :, None])[:, :, 0]
        Cn = Cp - Kg @ Cp[:, :2, :]
        dchi = (r[:, None, :] @ Si @ r[:, :, None])[:, 0, 0]
        am = act[:, None]
        p = torch.where(am, pn, p)
        C = torch.where(am[:, :, None], Cn, C)
        chi2 = chi2 + torch.where(act, dchi, torch.zeros_like(dchi))
    return chi2.sum()


def map_gradient(map_np: np.ndarray, seeds: dict, y, z, row_x, include=None, **prm):
    """(loss, d loss / d map) in float64 by reverse-mode autograd."""
    m = torch.tensor(np.asarray(map_np, np.float64), requires_grad=True)
    fitprm = {k: prm[k] for k in ("bz", "sigma_y", "sigma_z", "var_sin0", "var_tgl0", "var_qpt0")}
    L = chi2_sum_torch(m, seeds, y, z, row_x, include=include, **fitprm)
    L.backward()
    return float(L.detach()), m.grad.numpy().copy()
