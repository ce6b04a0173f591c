"""Algorithmic HBM traffic of the solver's kernels: every vector element a
kernel must read or write, counted once (halo re-reads served by cache are
not counted).  Used to turn measured times into achieved bandwidth.

Per-unknown figures for one level with n unknowns, element size e bytes
(8 for FP64, 4 for the FP32 preconditioner):

  line-relaxation half-sweep, u = 0 on entry   : own b read, own u write      = e      per unknown of the level
  line-relaxation half-sweep                   : own b, other-colour u, own u = 1.5 e
  residual + restriction (colour-1 residual 0) : b red, u both, coarse write  = 1.75 e
  prolongation + add (colour-0 columns only)   : u red r/w, coarse read      = 1.25 e
  CG operator + <p,q>                          : p read, q write              = 16 B
  CG update u, r                               : u, p, r, q read; u, r write  = 48 B
  CG dots <r,z>, <z,q>                         : r, z, q read                 = 16 B + z size
  CG direction p = z + beta p                  : z, p read; p write           = 16 B + z size
"""
from __future__ import annotations


def smooth_bytes(n: int, e: int, zero: bool) -> float:
    return n * (e if zero else 1.5 * e)


def vcycle_bytes(n0: int, levels: int, e: int, nu_pre=1, nu_post=1, nu_coarse=1) -> float:
    """Bytes of one V-cycle with rho = 1 (the shortcuts of the schedule)."""
    total = 0.0
    n = n0
    for l in range(levels):
        if l == levels - 1:
            if nu_coarse > 0:
                total += smooth_bytes(n, e, True) + smooth_bytes(n, e, False)
                total += (nu_coarse - 1) * 2 * smooth_bytes(n, e, False)
        else:
            if nu_pre > 0:
                total += smooth_bytes(n, e, True) + smooth_bytes(n, e, False)
                total += (nu_pre - 1) * 2 * smooth_bytes(n, e, False)
            total += 1.75 * e * n                      # residual + restriction
            total += 1.25 * e * n                      # prolongation (red only)
            total += nu_post * 2 * smooth_bytes(n, e, False)
        n //= 4
    return total


def pcg_iteration_bytes(n0: int, levels: int, e: int, **mg) -> float:
    z = e
    cg = 16 * n0 + 48 * n0 + (16 + z) * n0 + (16 + z) * n0
    cast = (8 + 4) * n0 if e == 4 else 0.0
    return cg + cast + vcycle_bytes(n0, levels, e, **mg)


def smooth0_launch_bytes(n0: int, e: int, nu_pre=1, nu_post=1) -> float:
    """Average algorithmic bytes of one finest-level half-sweep launch in a
    V-cycle (the first pre-smoothing sweep starts from u = 0)."""
    launches = 2 * nu_pre + 2 * nu_post
    total = smooth_bytes(n0, e, True) + (launches - 1) * smooth_bytes(n0, e, False)
    return total / launches
