"""The seeded input generators: lattice chains are valid, and the drawn
workloads do not change silently (checksums of the arrays both the oracle and
the HIP library consume)."""
import hashlib

import numpy as np
import pytest

from paper_1705_02180_amd import inputs as I


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


@pytest.mark.parametrize("n,seed", [(20, 1), (343, 2), (1601, 3)])
def test_compact_native_is_a_self_avoiding_lattice_walk(n, seed):
    x = I.compact_native(n, seed).T / I.LATTICE
    q = np.rint(x - x[0]).astype(np.int64)
    assert np.allclose(x - x[0], q, atol=1e-9)                # on the lattice
    steps = np.abs(np.diff(q, axis=0)).sum(axis=1)
    assert np.all(steps == 1)                                  # unit lattice bonds
    assert len({tuple(r) for r in q}) == n                     # self-avoiding
    ext = q.max(axis=0) - q.min(axis=0) + 1
    assert np.prod(ext) <= 2 * n + 8                           # compact: fills its box


def test_persistent_start_is_self_avoiding_with_jitter():
    x = I.persistent_start(1000, 5).T
    d = np.linalg.norm(np.diff(x, axis=0), axis=1)
    assert np.all(np.abs(d - I.LATTICE) < 0.5)
    q = np.rint((x - x[0]) / I.LATTICE)
    assert len({tuple(r) for r in q}) == 1000


def test_generated_inputs_are_unchanged():
    w = I.config2(n_replicas=2)
    s = w.systems[0]
    assert [digest(s.native), digest(s.start), digest(s.charge), digest(s.mass), digest(s.contact_idx)] == [
        "e07146f6e1a7ae67", "b944751fc1b8e9b9", "7a1420b0274a8f4e", "cf45165bd69eb38d", "6bd267a6dbf50fff"]
    w = I.config1(n_replicas=2)
    assert [digest(w.systems[0].native), digest(w.systems[0].start)] == ["8ebbb67bbf080f07", "7b8d1240829e17c3"]
    assert digest(I.compact_native(1601, 7)) == "656b99f75a60e9ad"
    assert digest(I.persistent_start(3000, 8)) == "9d63c207b17f021f"


def test_cutoff_workload_starts_compact_without_overlaps():
    w = I.config6(n_replicas=3, n=600)
    assert w.params["r_cut_contact"] == 12.0 and w.params["r_cut_nb"] == 12.0 and w.params["bias_mode"] == 0
    X = w.initial_x().reshape(3, 3, 600)
    nat = w.systems[0].native
    assert np.abs(X - nat[None]).max() < 0.5                     # jittered native
    assert not np.array_equal(X[0], X[1])                        # one draw per replica
    d = np.sqrt(((X[1][:, :, None] - X[1][:, None, :]) ** 2).sum(0).astype(np.float64))
    np.fill_diagonal(d, np.inf)
    assert d.min() > 3.0                                         # lattice spacing 3.8 A minus the jitter
