"""The C-ABI library loads and exports every entry point include/scps.h
declares, and rejects bad arguments on the host before touching the GPU.
No call here launches device work."""
import ctypes as C
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scps.h")
LIB = os.environ.get("SCPS_LIB") or os.path.join(ROOT, "paper_1705_02180_amd", "libscps.so")


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
    for mode in (4, 3):                   # no such mode; the overlapped schedule without SCPS bias
        with pytest.raises(scps.ScpsError) as e:
            scps.Context.from_workload(w, exec_mode=mode)
        assert e.value.status == -1, mode
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
    assert lib.scps_set_launch(None, 2, 4) == -1
    assert lib.scps_get_launch(None, None) == -1
    assert lib.scps_set_graph_steps(None, 16) == -1
    assert lib.scps_eval_zbias(None, None, None, None, None, None) == -1
    assert lib.scps_zbias_backward(None, None, None, None, C.c_int64(0), None, C.c_int64(0), None, None) == -1
    lib.scps_last_error.restype = C.c_char_p
    assert b"NULL" in lib.scps_last_error()


def test_context_free_entry_points_validate_on_the_host(lib):
    """The toy-model and convergence-measure calls need no context; bad
    arguments come back as status codes before any device work."""
    from paper_1705_02180_amd import inputs as I
    from paper_1705_02180_amd import scps
    D = C.c_double(0.0)
    fake = C.c_void_p(0x1000)              # never dereferenced: validation fails first
    f = lib.scps_path_distance
    f.restype = C.c_int
    f.argtypes = scps._lib.scps_path_distance.argtypes
    assert f(None, 5, fake, 5, 0.0, 0.0, 0.8, 20, 20, None, C.byref(D)) == -1     # NULL points with n > 0
    assert f(fake, 5, fake, 5, 0.0, 0.0, 0.0, 20, 20, None, C.byref(D)) == -1     # cell <= 0
    assert f(fake, 5, fake, 5, 0.0, 0.0, 0.8, 0, 20, None, C.byref(D)) == -1      # empty grid
    g = lib.scps_path_distance_noalloc                                           # the variant without allocation
    g.restype = C.c_int
    g.argtypes = scps._lib.scps_path_distance_noalloc.argtypes
    assert g(None, 5, fake, 5, 0.0, 0.0, 0.8, 20, 20, None, C.byref(D)) == -1
    assert g(fake, 5, fake, 5, 0.0, 0.0, -1.0, 20, 20, None, C.byref(D)) == -1
    assert g(fake, 5, fake, 5, 0.0, 0.0, 0.8, 1025, 1024, None, C.byref(D)) == -2   # beyond its 2^20 cells
    fs = lib.scps_funnel_steps
    fs.restype = C.c_int
    fs.argtypes = scps._lib.scps_funnel_steps.argtypes
    p = I.funnel_params()
    fp = scps.FunnelParams(A1=p["A1"], A2=p["A2"], A3=p["A3"], s1=p["s1"], s2=p["s2"], s3=p["s3"], w=p["w"],
                           xm=p["xm"], ym=p["ym"], kT=p["kT"], mobility_dt=p["mob_dt"], bias_mode=1, w_form=0,
                           k_R=p["k_R"], lam=p["lam"], k_s=p["k_s"], k_w=p["k_w"], seed=1)
    assert fs(None, 4, 0, fake, fake, 1, 0, 0, None, 0, None, None) == -1             # no parameters
    assert fs(C.byref(fp), 4, 0, fake, fake, 1, 0, 0, None, 10, None, None) == -1      # no mean path
    assert fs(C.byref(fp), 4, 0, fake, fake, 1, 0, 0, None, 129, fake, None) == -2     # 129 frames
    assert fs(C.byref(fp), 0, 0, fake, fake, 1, 0, 0, None, 10, fake, None) == -1      # no trajectory
    assert fs(C.byref(fp), 4, 0, fake, fake, 1, 0, 5, None, 10, fake, None) == -1      # frames NULL
    fm = lib.scps_funnel_mean_path
    fm.restype = C.c_int
    fm.argtypes = scps._lib.scps_funnel_mean_path.argtypes
    zeros = (C.c_uint8 * 4)()
    assert fm(4, 3, fake, zeros, fake, None) == -7                                    # no successful trajectory
    assert fm(4, 3, None, zeros, fake, None) == -1


def test_init_lays_out_every_chain_shape_before_device_memory(lib):
    """scps_init_system builds the host-side layout (internal particle order,
    tile flags and sub-step masks, the persistent schedules, the per-step
    work lists) before its first device allocation.  Several chain shapes run
    through it: two particles, a ragged chain with a partial contact set,
    min_seq_sep 35 on the heavy-particle contact set, both cutoffs (the
    neighbour-list path), two systems of different lengths, SCPS mode.  With a
    GPU every context is created and destroyed; without one each call stops
    at the first device allocation with a HIP status and frees what it held.
    (Under tests/run_sanitizers.sh this puts that host code under ASan and
    UBSan.)"""
    import torch
    from paper_1705_02180_amd import inputs as I
    from paper_1705_02180_amd import scps
    base = dict(I._base_params())
    w2 = I.config2(n_replicas=3, n_steps=1)
    cases = [   # params, chain lengths, contact sets, replica systems, exec mode
        (base, [2], [[0, 1]], [0], 0),
        (dict(base, min_seq_sep=5), [257], [list(range(0, 257, 3))], [0, 0], 0),
        (dict(w2.params, min_seq_sep=35), [560], [w2.systems[0].contact_idx], [0, 0, 0], 0),
        (dict(base, r_cut_contact=12.0, r_cut_nb=12.0), [300], [list(range(300))], [0, 0], 1),
        (dict(base, bias_mode=1), [150, 200], [list(range(150)), list(range(0, 200, 2))], [0, 1, 1, 0], 0),
        (dict(base, bias_mode=1), [130], [list(range(130))], [0] * 40, 2),
    ]
    for p, sizes, cidx, rsys, exec_mode in cases:
        mass = [np.full(n, 1.0, np.float32) for n in sizes]
        charge = [np.zeros(n, np.float32) for n in sizes]
        try:
            ctx = scps.Context(p, sizes, cidx, mass, charge, rsys, exec_mode=exec_mode)
        except scps.ScpsError as e:
            assert not torch.cuda.is_available() and e.status == -4, (sizes, e)
        else:
            assert torch.cuda.is_available()
            ctx.close()
