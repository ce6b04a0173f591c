"""Kernel timing through the C ABI: ell_profile_enable records HIP events on
the launch stream around each finest-level half-sweep, ell_profile_pause
stops and resumes the recording without dropping what was recorded (a
benchmark times a sample of its steps that way)."""
import numpy as np
import pytest
import torch

from paper_1307_2036_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ell():
    from paper_1307_2036_amd import ell as E
    E.load_library()
    assert torch.cuda.is_available()
    return E


def test_profile_pause_and_resume(ell):
    p = I.config0()
    G = ell.Grid.from_problem(p)
    assert G.levels >= 2
    r = torch.from_numpy(np.ascontiguousarray(p.f)).cuda()
    fam = ell.ELL_K_SMOOTH0
    per_cycle = 2 * p.nu_pre + 2 * p.nu_post  # finest-level half-sweeps of one V-cycle
    G.profile_enable(fam, 3 * per_cycle)
    G.profile_pause(fam, True)
    G.vcycle(r)
    assert G.profile_read(fam)[0] == 0
    G.profile_pause(fam, False)
    G.vcycle(r)
    n, ms = G.profile_read(fam)
    assert n == per_cycle and ms > 0.0
    t = G.profile_times(fam)
    assert t.shape == (per_cycle,) and np.all(t > 0.0)
    G.profile_pause(fam, True)
    G.vcycle(r)
    assert G.profile_read(fam)[0] == per_cycle
    # resumed, the recording stops at the capacity
    G.profile_pause(fam, False)
    for _ in range(3):
        G.vcycle(r)
    assert G.profile_read(fam)[0] == 3 * per_cycle
    # enabling again starts a new, running record
    G.profile_pause(fam, True)
    G.profile_enable(fam, per_cycle)
    G.vcycle(r)
    assert G.profile_read(fam)[0] == per_cycle
    G.close()


def test_profile_arguments_are_checked(ell):
    p = I.config0()
    G = ell.Grid.from_problem(p)
    with pytest.raises(ell.EllError):
        G.profile_pause(ell.ELL_K_COUNT, True)
    with pytest.raises(ell.EllError):
        G.profile_enable(-1, 4)
    G.close()
