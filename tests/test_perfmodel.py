"""The algorithmic byte model behind the roofline figures (bytes every kernel
must read or write once, per unknown of the level): the per-kernel figures
and their sums at 512 x 512 x 128, written out from the arrays each kernel
touches."""
import pytest

from paper_1307_2036_amd import perfmodel as P

N = 512 * 512 * 128


def test_half_sweeps():
    # first sweep from zero: own b read, own u written (half the level each): e;
    # later: own b, the other colour's u, own u: 1.5 e
    assert P.smooth_bytes(N, 8, True) == 8 * N
    assert P.smooth_bytes(N, 8, False) == 12 * N
    assert P.smooth_bytes(N, 4, False) == 6 * N


def test_finest_launch_average():
    # (8 + 12 + 12 + 12) / 4 = 11 B plain; the fused update adds q read and r
    # write over the first pair (16), the fused prolongation the coarse read
    # (2) and colour 1 of r on the last sweep (4): (16 + 20 + 14 + 16) / 4
    assert P.smooth0_launch_bytes(N, 8) == 11 * N
    assert P.smooth0_launch_bytes(N, 8, fused_update=True, fused_prolong=True) == pytest.approx(16.5 * N)


def test_vcycle_and_iteration():
    # four levels, five coarse sweep pairs: 91.0625 B per fine unknown;
    # the coarse-level fused prolongations save 1 e per unknown of levels 1, 2
    assert P.vcycle_bytes(N, 4, 8, nu_coarse=5) == pytest.approx(91.0625 * N)
    assert P.vcycle_bytes(N, 4, 8, nu_coarse=5, coarse_prolong=True) == pytest.approx(
        (91.0625 - 8 * (1 / 4 + 1 / 16)) * N)
    assert P.pcg_iteration_bytes(N, 4, 8, nu_coarse=5) == pytest.approx(183.0625 * N)
    assert P.hybrid_vcycle_bytes(N, 4, 5) == pytest.approx(65.53125 * N)
    # mixed precision with the fused prolongation: the 7 B pass goes, the
    # first FP64 post-sweep reads 3 B of FP32 values for 4 B of FP64 ones
    assert P.hybrid_vcycle_bytes(N, 4, 5, fused_prolong=True) == pytest.approx(57.53125 * N)
    assert P.smooth0_launch_bytes_hybrid(N) == pytest.approx(9.5 * N)
    assert P.smooth0_launch_bytes_hybrid(N, fused_prolong=True) == pytest.approx(9.25 * N)
    # and on the FP32 levels 1, 2: 1 e = 4 B per unknown of those levels
    assert P.hybrid_vcycle_bytes(N, 4, 5, fused_prolong=True, coarse_prolong=True) == pytest.approx(
        (57.53125 - 4 * (1 / 4 + 1 / 16)) * N)


def test_cg_vector_work():
    # operator step 44 (32 + deferred updates 12 on average), residual update
    # 24 (16 fused), dots 24 / 16 (flexible / classic; 8 / 0 fused)
    assert P.cg_bytes(N, True) == 92 * N
    assert P.cg_bytes(N, False) == 84 * N
    assert P.cg_bytes(N, False, fused_update=True, fused_dots=True) == 60 * N


def test_varying_fields():
    # a half-sweep reads its colour's faces, 1/p and T/p: 12 B per unknown of the level
    assert P.smooth_bytes_varying(N, False) == 24 * N
    assert P.smooth0_launch_bytes_varying(N) == pytest.approx(23 * N)
    assert P.smooth0_launch_bytes_varying_hybrid(N) == pytest.approx(18.5 * N)
