"""Applying solved controls to a higher-resolution image (Sec. 4.3).

Positions are normalised to [0,1]^2 (Def. 3.1), so a control eps(t) found on
one grid applies unchanged to a finer grid of the same scene; only one
forward sweep is needed.  With the windowed sum the pixel radius grows with
the resolution (R -> f R) and the normalisation s shrinks by f^2, so that
every agent still averages over the same physical neighbourhood with the
same weight per unit area.
"""
from __future__ import annotations

from .binding import Params, abc_forward_dynamics


def transfer_params(p: Params, H_lo: int, W_lo: int, factor: int) -> Params:
    """Parameters for a grid `factor` times finer per side than H_lo x W_lo."""
    if factor < 1:
        raise ValueError("factor must be >= 1")
    s_lo = p.inv_norm if p.inv_norm > 0 else 1.0 / min(H_lo * W_lo, (2 * p.R + 1) ** 2)
    return p.replace(R=p.R * factor, inv_norm=s_lo / factor ** 2, ckpt_every=max(p.ckpt_every, 0))


def transfer(c_hi, eps, p_lo: Params, H_lo: int, W_lo: int, factor: int):
    """c(T) of the finer image under the coarse grid's controls (one forward sweep)."""
    ph = transfer_params(p_lo, H_lo, W_lo, factor)
    return abc_forward_dynamics(c_hi, eps, ph)[-1]
