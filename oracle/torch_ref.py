"""Vectorised FP64 PyTorch-CPU restatement of the explicit time loop.

TEST INFRASTRUCTURE ONLY.  It exists to cross-check the C oracle's hand-written
adjoint with torch autograd: it states the same method (eq. (3) / Algorithm 1
for the transformation, Scheme 1 for diffusion, transformation first as in
Sec. III) with whole-array operations instead of loops, and shares no code
with either the C oracle or the HIP path.  Everything runs on the CPU in
float64.
"""
from __future__ import annotations

import torch

RATE_NAMES = ("v_dom", "k_dom", "rho", "mu", "beta", "v_som", "v_p4")


def transform(x: torch.Tensor, r: dict, dt: float, mort_to_p4: bool = False) -> torch.Tensor:
    """Eq. (3) with the clamps of Algorithm 1.  x: [5, n]; r: rate tensors."""
    x1, x2, x3, x4, x5 = x[0], x[1], x[2], x[3], x[4]
    uptake = r["v_dom"] * x2 / (r["k_dom"] + x2) * x1 * dt
    uptake = torch.where(uptake > x2, x2, uptake)
    resp = r["rho"] * x1 * dt
    morta = r["mu"] * x1 * dt
    over = resp + morta > x1
    all_dies = morta > x1
    new_morta = torch.where(over & all_dies, x1, morta)
    new_resp = torch.where(over, torch.where(all_dies, torch.zeros_like(resp), x1 - morta), resp)
    morta, resp = new_morta, new_resp
    if mort_to_p4:
        m_dom, m_som, m_p4 = 0.0 * morta, 0.0 * morta, morta
    else:
        m_dom, m_som, m_p4 = r["beta"] * morta, (1.0 - r["beta"]) * morta, 0.0 * morta
    t_fom = r["v_p4"] * x4 * dt
    t_fom = torch.where(t_fom > x4, x4, t_fom)
    t_som = r["v_som"] * x3 * dt
    t_som = torch.where(t_som > x3, x3, t_som)
    return torch.stack([
        x1 + uptake - morta - resp,
        x2 + m_dom - uptake + t_fom + t_som,
        x3 + m_som - t_som,
        x4 + m_p4 - t_fom,
        x5 + resp,
    ])


def diffuse(x: torch.Tensor, nbr: torch.Tensor, w: torch.Tensor, D: torch.Tensor, dt: float,
            h: float) -> torch.Tensor:
    """Scheme 1 for all five pools: x_s + (D_s dt / h^2) * sum_j w_ij (x_s,j - x_s,i)."""
    present = nbr >= 0
    j = torch.where(present, nbr, torch.zeros_like(nbr)).long()
    out = []
    for s in range(5):
        m = x[s]
        diffs = torch.where(present, m[j] - m.unsqueeze(0), torch.zeros_like(w))
        out.append(m + D[s] * dt / (h * h) * (w * diffs).sum(0))
    return torch.stack(out)


def totals(x: torch.Tensor, seg_off) -> torch.Tensor:
    """[nseg][5] pool sums per volume."""
    return torch.stack([x[:, int(seg_off[g]):int(seg_off[g + 1])].sum(1)
                        for g in range(len(seg_off) - 1)])


def run_totals(x0: torch.Tensor, nbr: torch.Tensor, region: torch.Tensor, c: torch.Tensor,
               D: torch.Tensor, r: dict, dt: float, h: float, nsteps: int, seg_off,
               order: int = 0, mort_to_p4: bool = False) -> torch.Tensor:
    """Totals after every step ([nsteps+1][nseg][5]) with w_ij = (c_r(i) + c_r(j)) / 2."""
    present = nbr >= 0
    j = torch.where(present, nbr, torch.zeros_like(nbr)).long()
    w = torch.where(present, 0.5 * (c[region.long()].unsqueeze(0) + c[region.long()][j]),
                    torch.zeros(nbr.shape, dtype=torch.float64))
    x = x0
    out = [totals(x, seg_off)]
    for _ in range(nsteps):
        if order == 0:
            x = diffuse(transform(x, r, dt, mort_to_p4), nbr, w, D, dt, h)
        else:
            x = transform(diffuse(x, nbr, w, D, dt, h), r, dt, mort_to_p4)
        out.append(totals(x, seg_off))
    return torch.stack(out)


def run_state(x0, nbr, region, c, D, r, dt, h, nsteps, order=0, mort_to_p4=False):
    """Final state after ``nsteps`` steps."""
    present = nbr >= 0
    j = torch.where(present, nbr, torch.zeros_like(nbr)).long()
    w = torch.where(present, 0.5 * (c[region.long()].unsqueeze(0) + c[region.long()][j]),
                    torch.zeros(nbr.shape, dtype=torch.float64))
    x = x0
    for _ in range(nsteps):
        if order == 0:
            x = diffuse(transform(x, r, dt, mort_to_p4), nbr, w, D, dt, h)
        else:
            x = transform(diffuse(x, nbr, w, D, dt, h), r, dt, mort_to_p4)
    return x
