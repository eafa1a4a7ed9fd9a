"""The C-ABI library loads and exports every entry point include/scps.h
declares, and rejects bad arguments on the host before touching the GPU.
No call here launches device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scps.h")
LIB = os.path.join(ROOT, "paper_1705_02180_amd", "libscps.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scps_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)
    if not os.path.exists(LIB):
        from paper_1705_02180_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("scps_init_system", "scps_set_reference_map", "scps_step_replicas",
                 "scps_eval_z_and_grad", "scps_update_reference_from_paths"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_names_match_header(lib):
    from paper_1705_02180_amd import scps
    assert sorted(scps.EXPORTS) == declared_symbols()


def test_host_validation_rejects_bad_arguments(lib):
    from paper_1705_02180_amd import inputs as I
    from paper_1705_02180_amd import scps
    w = I.config1(n_replicas=2, n_steps=1)
    bad = [dict(integrator=7), dict(bias_mode=3), dict(dt=0.0), dict(nb_excl=0), dict(r0_contact=-1.0)]
    for b in bad:
        p = dict(w.params)
        p.update(b)
        with pytest.raises(scps.ScpsError) as e:
            scps.Context.from_workload(w, params=p)
        assert e.value.status == -1, b
    with pytest.raises(scps.ScpsError) as e:
        scps.Context(w.params, [20], [[3, 2]], [w.systems[0].mass], [w.systems[0].charge], [0])
    assert e.value.status == -1
    with pytest.raises(scps.ScpsError) as e:
        scps.Context(w.params, [20], [[1, 2]], [w.systems[0].mass], [w.systems[0].charge], [1])
    assert e.value.status == -1
    with pytest.raises(scps.ScpsError) as e:      # one grid row per replica
        scps.Context(w.params, [20], [[1, 2]], [w.systems[0].mass], [w.systems[0].charge], [0] * 65536)
    assert e.value.status == -2
    assert lib.scps_step_replicas(None, None, None, None, C.c_int64(1), C.c_uint64(0), 0, None) == -1
    lib.scps_last_error.restype = C.c_char_p
    assert b"NULL" in lib.scps_last_error()
