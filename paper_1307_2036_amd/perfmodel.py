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
  CG dots <r,z>, <z,q> (flexible beta)         : r, z, q read                 = 16 B + z size
  CG dot <r,z> (classic beta)                  : r, z read                    = 8 B + z size
  CG direction p = z + beta p                  : z, p read; p write           = 16 B + z size
"""
from __future__ import annotations


def smooth_bytes(n: int, e: int, zero: bool) -> float:
    return n * (e if zero else 1.5 * e)


def vcycle_bytes(n0: int, levels: int, e: int, nu_pre=1, nu_post=1, nu_coarse=1, coarse_prolong=False,
                 pro_from=1) -> float:
    """Bytes of one V-cycle with rho = 1 (the shortcuts of the schedule).
    coarse_prolong: on levels pro_from .. levels - 2 the prolongation rides on
    the first post-smoothing sweep, which reads the coarse correction (0.25 e
    per unknown of the level) instead of the 1.25 e of the pass."""
    total = 0.0
    n = n0
    for l in range(levels):
        if l == levels - 1:
            if nu_coarse > 0:
                total += smooth_bytes(n, e, True) + smooth_bytes(n, e, False)
                total += (nu_coarse - 1) * 2 * smooth_bytes(n, e, False)
            else:  # no coarse sweeps: pre and post sweeps without a coarser correction
                if nu_pre > 0:
                    total += smooth_bytes(n, e, True) + smooth_bytes(n, e, False)
                    total += (nu_pre - 1) * 2 * smooth_bytes(n, e, False)
                total += nu_post * 2 * smooth_bytes(n, e, False)
        else:
            if nu_pre > 0:
                total += smooth_bytes(n, e, True) + smooth_bytes(n, e, False)
                total += (nu_pre - 1) * 2 * smooth_bytes(n, e, False)
            total += 1.75 * e * n                      # residual + restriction
            total += (0.25 if coarse_prolong and l >= pro_from else 1.25) * e * n  # prolongation (red only)
            total += nu_post * 2 * smooth_bytes(n, e, False)
        n //= 4
    return total


def cg_bytes(n0: int, flexible: bool = True, fused_update: bool = False, fused_dots: bool = False) -> float:
    """CG vector work per iteration (FP64) beyond the V-cycle's own bytes:
    fused direction + operator (z, p_old read; p_new, q written: 32 B) and the
    deferred solution updates, two at a time on every other iteration (u,
    p_old2 read, u written: 24 B per two iterations, 12 B on average: 44 B);
    residual update (r, q read, r written: 24 B; on
    the first pre-smoothing pair, which reads r anyway: q read, r written,
    16 B); dots <r,z>, <z,q> (24 B; <r,z> alone, 16 B, with the classic beta; on
    the last post-smoothing pair: nothing, or the q read, 8 B, for <z,q>)."""
    update = 16 if fused_update else 24
    if fused_dots:
        dots = 8 if flexible else 0
    else:
        dots = 24 if flexible else 16
    return (44 + update + dots) * n0


def hybrid_vcycle_bytes(n0: int, levels: int, nu_coarse=1, fused_prolong=False, coarse_prolong=False) -> float:
    """Mixed-precision V-cycle: FP32 everywhere except the finest level, whose
    pre-smoothing and restriction read the FP64 residual and write FP32, and
    whose colour-0 prolongation and post-smoothing write the FP64 output.
    fused_prolong: no prolongation pass; the first FP64 post-sweep reads the
    FP32 colour-0 values and the coarse correction (3 B) in place of the FP64
    colour-0 values (4 B); coarse_prolong: the same on the FP32 levels 1 ..
    levels - 2 (vcycle_bytes)."""
    fine = (6 + 8) * n0          # pre red (b64 read, u32 write), pre black (+ u32 red read)
    fine += (4 + 4 + 1) * n0     # restriction: b64 red, u32 both colours, coarse write
    if fused_prolong:
        fine += (4 + 2 + 1 + 4) * n0 + 12 * n0  # post black (r, u32 red, coarse, z), post red
    else:
        fine += (2 + 1 + 4) * n0     # prolongation: u32 red, coarse, z64 red write
        fine += 2 * 12 * n0          # FP64 post-smoothing, black then red
    return fine + vcycle_bytes(n0 // 4, levels - 1, 4, nu_coarse=nu_coarse, coarse_prolong=coarse_prolong,
                               pro_from=0)


def pcg_iteration_bytes(n0: int, levels: int, e: int, nu_coarse=1, flexible=True, fused_update=False,
                        fused_dots=False, fused_prolong=False, coarse_prolong=False, **mg) -> float:
    """fused_prolong: the finest prolongation (10 B/unknown) rides on the first
    post-smoothing sweep, which reads the coarse correction (2 B/unknown), and
    the last sweep reads colour 1 of r for <r, z> (4 B/unknown); coarse_prolong:
    the same on the coarse levels (vcycle_bytes).  e = 4: the mixed-precision
    V-cycle (hybrid_vcycle_bytes, its own fused prolongation)."""
    cg = cg_bytes(n0, flexible, fused_update, fused_dots)
    if e == 8:
        return (cg + vcycle_bytes(n0, levels, 8, nu_coarse=nu_coarse, coarse_prolong=coarse_prolong, **mg) -
                (4 * n0 if fused_prolong else 0))
    return cg + hybrid_vcycle_bytes(n0, levels, nu_coarse, fused_prolong, coarse_prolong)


def smooth0_launch_bytes_hybrid(n0: int, fused_update: bool = False, dot_q: bool = False,
                                fused_prolong: bool = False) -> float:
    """Average bytes of a finest-level half-sweep launch in the mixed-precision
    V-cycle: FP32 pre-sweeps reading the FP64 residual, FP64 post-sweeps; with
    the fused residual update the pre-sweeps also read q and write r (16 B per
    unknown of their colour), with the fused <z,q> the post-sweeps read q; with
    the fused prolongation the first post-sweep reads the FP32 colour-0 values
    and the coarse correction (3 B) in place of the FP64 ones (4 B)."""
    post = (11 if fused_prolong else 12) + 12
    return ((6 + 8 + post) + (16 if fused_update else 0) + (8 if dot_q else 0)) * n0 / 4


def smooth0_launch_bytes(n0: int, e: int, nu_pre=1, nu_post=1, fused_update: bool = False,
                         dot_q: bool = False, fused_prolong: bool = False) -> float:
    """Average algorithmic bytes of one finest-level half-sweep launch in a
    V-cycle (the first pre-smoothing sweep starts from u = 0).  The fused
    residual update adds the q read and the r write to the first pre-smoothing
    pair (8 + 8 B per unknown of each colour), the fused <z,q> the q read to the
    last post-smoothing pair, the fused prolongation the coarse correction
    (2 B per fine unknown) to the first post-smoothing sweep and colour 1 of r
    (4 B) to the last."""
    launches = 2 * nu_pre + 2 * nu_post
    total = smooth_bytes(n0, e, True) + (launches - 1) * smooth_bytes(n0, e, False)
    total += (16 * n0 if fused_update else 0) + (8 * n0 if dot_q else 0) + (6 * n0 if fused_prolong else 0)
    return total / launches


# ---------------------------------------------------------------------------
# horizontally varying vertical coefficients (FP64, per-column fields): every
# half-sweep also reads its colour's faces, 1/p and T/p (24 B per unknown of
# the colour = 12 B per unknown of the level); the restriction reads the faces
# of the colour-0 children (4 B); the CG operator step the faces (8 B)
# ---------------------------------------------------------------------------
def smooth_bytes_varying(n: int, zero: bool) -> float:
    return smooth_bytes(n, 8, zero) + 12 * n


def smooth0_launch_bytes_varying(n0: int, nu_pre=1, nu_post=1, fused_update=False, dot_q=False) -> float:
    """Average algorithmic bytes of one finest-level half-sweep launch (the
    fused residual update adds the q read and the r write to the first pair,
    the fused <z, q> the q read to the last, as in smooth0_launch_bytes)."""
    launches = 2 * nu_pre + 2 * nu_post
    total = smooth_bytes_varying(n0, True) + (launches - 1) * smooth_bytes_varying(n0, False)
    total += (16 * n0 if fused_update else 0) + (8 * n0 if dot_q else 0)
    return total / launches


def pcg_iteration_bytes_varying(n0: int, levels: int, nu_coarse=1, flexible=True, nu_pre=1,
                                nu_post=1, fused_update=False, fused_dots=False) -> float:
    """One PCG iteration on a varying grid (cg_bytes for the fused forms)."""
    total = (cg_bytes(n0, flexible, fused_update, fused_dots) + 8 * n0 +
             vcycle_bytes(n0, levels, 8, nu_pre, nu_post, nu_coarse))
    n = n0
    for l in range(levels):
        if l == levels - 1:
            sweeps = 2 * (nu_coarse if nu_coarse > 0 else nu_pre + nu_post)
        else:
            sweeps = 2 * (nu_pre + nu_post)
            total += 4 * n
        total += sweeps * 12 * n
        n //= 4
    return total


def smooth0_launch_bytes_varying_hybrid(n0: int, fused_update=False, dot_q=False) -> float:
    """Average algorithmic bytes of a finest-level half-sweep launch of the
    mixed-precision V-cycle on a varying grid, per unknown of the level: the
    FP32 pre-sweeps read the FP64 residual (4 B), write FP32 u (2 B), the second
    reads the other colour (2 B), and each reads its colour's FP32 faces, 1/p
    and T/p (6 B); the FP64 post-sweeps read r (4 B) and the other colour of z
    (4 B), write z (4 B) and read the FP64 fields (12 B):
    (12 + 14 + 24 + 24) / 4 = 18.5 B; the fused forms add their q reads and r
    writes as in smooth0_launch_bytes_hybrid."""
    return ((12 + 14 + 24 + 24) + (16 if fused_update else 0) + (8 if dot_q else 0)) * n0 / 4


def pcg_iteration_bytes_varying_hybrid(n0: int, levels: int, nu_coarse=1, nu_pre=1, nu_post=1,
                                       fused_update=False, fused_dots=False) -> float:
    """One flexible PCG iteration on a varying grid with the mixed-precision
    V-cycle (separate residual update and dots): the FP64 CG work with the
    operator step's faces, the hybrid V-cycle, and the fields of every
    half-sweep (6 B per unknown of the level in FP32, 12 B for the FP64 finest
    post-sweeps) and restriction (2 B)."""
    total = cg_bytes(n0, True, fused_update, fused_dots) + 8 * n0 + hybrid_vcycle_bytes(n0, levels, nu_coarse)
    n = n0
    for l in range(levels):
        if l == levels - 1:
            sweeps = 2 * (nu_coarse if nu_coarse > 0 else nu_pre + nu_post)
            total += sweeps * 6 * n
        else:
            total += 2 * n + 2 * nu_pre * 6 * n + 2 * nu_post * (12 if l == 0 else 6) * n
        n //= 4
    return total
