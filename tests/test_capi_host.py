"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every
function include/lbm.h declares, and its pure host logic (sizes, velocity
tables, argument validation) behaves as documented."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2506_09242_amd import inputs, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_library_built_and_loads():
    assert os.path.exists(lbm.LIB_PATH), "run the build first"
    lbm.lib()


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # the binding knows every one of them, with a signature
    assert set(names) == set(lbm.SIGNATURES)


@pytest.mark.parametrize("q", [19, 27])
def test_velocity_table_matches_oracle_order(q):
    for i in range(q):
        c, w, o = lbm.lbm_velocity(q, i)
        c2, w2, o2 = oracle.velocity(q, i)
        assert tuple(c) == tuple(c2) and o == o2
        assert w == w2
    with pytest.raises(ValueError):
        lbm.lbm_velocity(q, q)


def test_population_bytes():
    for q, prec, s in [(19, lbm.LBM_F64, 8), (19, lbm.LBM_F32, 4), (27, lbm.LBM_F16S, 2)]:
        for dims in [(10, 7, 3), (64, 64, 1), (64, 64, 2), (100, 50, 9)]:
            cfg = lbm.make_config(*dims, q=q, prec=prec)
            N = dims[0] * dims[1] * dims[2]
            # whole blocks of 4096 nodes, Q slots each
            assert lbm.lbm_population_bytes(cfg) == -(-N // 4096) * 4096 * q * s
    bad = lbm.make_config(0, 1, 1)
    assert lbm.lbm_population_bytes(bad) == 0


def _create(cfg, tags):
    h = C.c_void_p()
    t = np.ascontiguousarray(tags, dtype=np.uint8)
    rc = lbm.lib().lbm_create(C.byref(cfg), t.ctypes.data_as(C.c_void_p), None, C.byref(h))
    return rc, h


@pytest.mark.parametrize("field,value,needle", [
    ("tau", 0.5, "tau"), ("tau", 0.3, "tau"), ("q", 15, "q must"), ("prec", 7, "precision"),
    ("rho0", 0.0, "rho0"), ("trt_lambda", -1.0, "trt_lambda"), ("smag_cs", -0.1, "smag_cs"),
    ("flags", 8, "flags"), ("flags", -1, "flags"), ("flags", 2, "multiples of 16"), ("flags", 6, "exclude"),
    ("nx", 0, "size"),
])
def test_create_rejects_bad_config(field, value, needle):
    cfg = lbm.make_config(4, 4, 4)
    setattr(cfg, field, value)
    rc, h = _create(cfg, inputs.all_fluid(4, 4, 4))
    assert rc == lbm.LBM_EINVAL and not h
    assert needle in lbm.lbm_last_error()


def test_create_rejects_bad_tags_and_fast_flows():
    cfg = lbm.make_config(4, 4, 4)
    t = inputs.all_fluid(4, 4, 4)
    t[1, 2, 3] = 12
    rc, _ = _create(cfg, t)
    assert rc == lbm.LBM_EINVAL and "unknown tag value 12" in lbm.lbm_last_error()
    # open boundaries: inlet only on x = 0, outlet only on x = nx-1, sane values
    t = inputs.all_fluid(4, 4, 4)
    t[0, 0, 1] = lbm.TAG_VIN
    rc, _ = _create(cfg, t)
    assert rc == lbm.LBM_EINVAL and "x = 0 plane" in lbm.lbm_last_error()
    t = inputs.all_fluid(4, 4, 4)
    t[0, 0, 0] = lbm.TAG_POUT
    rc, _ = _create(cfg, t)
    assert rc == lbm.LBM_EINVAL and "x = nx-1 plane" in lbm.lbm_last_error()
    t = inputs.all_fluid(4, 4, 4)
    t[:, :, 0] = lbm.TAG_VIN
    rc, _ = _create(lbm.make_config(4, 4, 4, bc_velocity=(0.4, 0, 0)), t)
    assert rc == lbm.LBM_EINVAL and "bc_velocity" in lbm.lbm_last_error()
    t = inputs.all_fluid(4, 4, 4)
    t[:, :, -1] = lbm.TAG_POUT
    rc, _ = _create(lbm.make_config(4, 4, 4, bc_density=(1.0, 0.0)), t)
    assert rc == lbm.LBM_EINVAL and "bc_density[1]" in lbm.lbm_last_error()
    t = inputs.all_fluid(4, 4, 4)
    t[:, :, 0] = lbm.TAG_PIN
    rc, _ = _create(lbm.make_config(4, 4, 4, bc_density=(-1.0, 1.0)), t)
    assert rc == lbm.LBM_EINVAL and "bc_density[0]" in lbm.lbm_last_error()
    t = inputs.all_fluid(4, 4, 4)
    t[0, 1, 2] = lbm.TAG_VOUT
    rc, _ = _create(cfg, t)
    assert rc == lbm.LBM_EINVAL and "x = nx-1 plane" in lbm.lbm_last_error()
    rc, _ = _create(cfg, np.zeros((4, 4, 4), np.uint8))
    assert rc == lbm.LBM_EINVAL and "no fluid" in lbm.lbm_last_error()
    cfg = lbm.make_config(4, 4, 4, force=(0.4, 0, 0))
    rc, _ = _create(cfg, inputs.all_fluid(4, 4, 4))
    assert rc == lbm.LBM_EINVAL and "force" in lbm.lbm_last_error()
    cfg = lbm.make_config(4, 4, 4, wall_velocity=[(0, 0, 0), (0.5, 0, 0)])
    rc, _ = _create(cfg, inputs.all_fluid(4, 4, 4))
    assert rc == lbm.LBM_EINVAL and "wall_velocity[1]" in lbm.lbm_last_error()
    cfg = lbm.make_config(2048, 1024, 1024)
    rc, _ = _create(cfg, np.zeros(1, np.uint8))
    assert rc == lbm.LBM_EINVAL and "2^31" in lbm.lbm_last_error()


def test_null_handles_are_rejected():
    L = lbm.lib()
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_set_launch(None, 64, 4) == lbm.LBM_EINVAL
    assert L.lbm_step_reduce_noalloc(None, 1, 1, None, 0) == lbm.LBM_EINVAL
    L.lbm_destroy(None)  # no-op
    assert L.lbm_time(None) == -1


def test_face_and_probe_argument_validation():
    L = lbm.lib()
    assert L.lbm_face_populations(19) == 5 and L.lbm_face_populations(27) == 9
    assert L.lbm_face_populations(0) == 0
    assert L.lbm_face_pack(None, 0, None) == lbm.LBM_EINVAL
    assert L.lbm_face_unpack(None, 1, None) == lbm.LBM_EINVAL
    # rejected before any device work
    assert L.lbm_probe_bandwidth(3, None, None, 4096 * 16, 16, None) == lbm.LBM_EINVAL
    assert "kind" in lbm.lbm_last_error()
    assert L.lbm_probe_bandwidth(0, None, None, 4096 * 16, 12, None) == lbm.LBM_EINVAL
    assert "lane_bytes" in lbm.lbm_last_error()
    assert L.lbm_probe_bandwidth(0, None, None, 4096 * 16 + 4, 16, None) == lbm.LBM_EINVAL
    assert "multiple" in lbm.lbm_last_error()
    assert L.lbm_probe_bandwidth(0, None, None, 4096 * 16, 16, None) == lbm.LBM_EINVAL
    assert "null" in lbm.lbm_last_error()


def test_mlp_argument_validation():
    L = lbm.lib()
    p = np.zeros(lbm.MLP_NPARAMS, np.float32)  # std entries 0: invalid
    rc = L.lbm_mlp_infer(p.ctypes.data_as(C.c_void_p), 0.01, None, 0, None, None)
    assert rc == lbm.LBM_EINVAL and "std" in lbm.lbm_last_error()
    assert L.lbm_mlp_train(None, None, None, 0, None, 0, 0, 0.0, None, None) == lbm.LBM_EINVAL
    assert L.lbm_mlp_grad(None, None, None, 0, None, None, None) == lbm.LBM_EINVAL


def test_header_compiles_as_c():
    """The header is plain C (no C++ constructs)."""
    r = subprocess.run(["gcc", "-std=c99", "-fsyntax-only", "-x", "c", HEADER], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

