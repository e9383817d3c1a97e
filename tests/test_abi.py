"""CPU-side checks of the C ABI: the library loads, exports every declared symbol,
and rejects bad shapes before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(pm_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    import paper_2410_20501_amd as pm
    lib = ctypes.CDLL(pm.hippm.LIB_PATH)
    declared = _declared()
    assert "pm_kdk" in declared and "pm_solve_mg" in declared
    for name in sorted(declared):
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    import paper_2410_20501_amd as pm
    assert _declared() <= set(pm.EXPORTED)


@pytest.mark.parametrize("n", [7, 6, 1026, 0, -4])
def test_create_rejects_bad_grid_without_a_device(n):
    import paper_2410_20501_amd as pm
    with pytest.raises(pm.PMError) as e:
        pm.Context(n)
    assert e.value.code == pm.PM_ERR_SHAPE


def test_create_rejects_unknown_flags_without_a_device():
    import paper_2410_20501_amd as pm
    with pytest.raises(pm.PMError) as e:
        pm.Context(16, 16, flags=8)
    assert e.value.code == pm.PM_ERR_ARG


def test_create_rejects_negative_particle_count():
    import paper_2410_20501_amd as pm
    with pytest.raises(pm.PMError) as e:
        pm.Context(32, -1)
    assert e.value.code == pm.PM_ERR_ARG


def test_struct_layouts_match_header():
    import paper_2410_20501_amd as pm
    assert ctypes.sizeof(pm.MGParams) == 40
    assert pm.MGParams.alpha.offset == 32
    assert pm.MGParams.cycle.offset == 36
    assert ctypes.sizeof(pm.MGStats) == 8 + 64 * 8
    assert pm.StepParams.mg.offset == 24
    assert pm.StepParams.timing.offset == 64
    assert pm.StepParams.omega_l.offset == 72
    assert pm.StepParams.gravity.offset == 80 and pm.StepParams.mond_family.offset == 84
    assert pm.StepParams.mond_param.offset == 112
    assert pm.StepParams.fr_f0.offset == 120 and pm.StepParams.fr_n.offset == 136
    assert pm.StepParams.fr_coarse_sweeps.offset == 156
    assert ctypes.sizeof(pm.StepParams) == 160
    p = pm.default_step_params()
    assert (p.mas, p.mg.pre, p.mg.post, p.mg.omega, p.mg.max_cycles) == (3, 2, 2, 1.0, 50)
    assert p.mg.alpha == 0.0 and p.mg.cycle == pm.PM_CYCLE_V
    assert p.omega_l == 0.0 and p.gravity == pm.PM_GRAVITY_NEWTON and p.mond_param == 1.0
    assert (p.fr_n, p.fr_cycles, p.fr_cycle, p.fr_pre, p.fr_post, p.fr_coarse_sweeps) == \
        (1, 1, pm.PM_CYCLE_F, 2, 1, 32)
    assert p.fr_f0 == -1e-5 and abs(p.fr_c2 - 29.9792458 ** 2) < 1e-9
