"""CPU-side checks of the C ABI: the library loads and exports every symbol the
header declares, and the header and binding agree on names and constants."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1602_06693_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pkm.h")


def _header_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pkm_[a-z0-9_]+)\s*\(", txt)))


def _header_defines():
    txt = open(HEADER).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (PKM_[A-Z0-9_]+)\s+(-?\d+)", txt)}


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpkm.so not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    declared = _header_functions()
    assert set(declared) == set(binding.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH],
                         capture_output=True, text=True).stdout
    for name in declared:
        assert re.search(rf"\bT {name}\b", out), name


def test_constants_match_header():
    for name, val in _header_defines().items():
        if name == "PKM_H":
            continue
        assert getattr(binding, name) == val, name


def test_version_string_loads_without_gpu():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpkm.so not built")
    assert "gfx950" in binding.pkm_version()


def test_null_context_is_rejected_without_gpu():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpkm.so not built")
    lib = binding.load()
    assert lib.pkm_kernel_mvm(None, None, 1, 0, None, None) == binding.PKM_ERR_INVALID
    assert lib.pkm_create(None, 0, None) == binding.PKM_ERR_INVALID
    assert b"NULL" in lib.pkm_last_error(None)


def test_adagrad_step_host_logic_matches_oracle():
    """pkm_adagrad_step is host-only: checked on the CPU against the oracle."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpkm.so not built")
    import numpy as np
    from oracle.adagrad import Adagrad
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(10)
    G = np.zeros(10)
    ref = Adagrad(eta=0.7)
    th_ref = theta.copy()
    for _ in range(5):
        g = rng.standard_normal(10)
        binding.pkm_adagrad_step(theta, g, G, eta=0.7)
        th_ref = ref.step(th_ref, g)
    assert np.allclose(theta, th_ref, rtol=1e-14, atol=1e-14)
    bad = np.array([1.0, np.nan])
    with pytest.raises(binding.PkmError):
        binding.pkm_adagrad_step(np.zeros(2), bad, np.zeros(2))


def test_tune_cache_rejects_shapes_the_library_does_not_instantiate(tmp_path):
    """A cached launch shape is used only if the launchers instantiate it for
    its key: FP16x3 keys (s4 >= 100) take 2 or 4 i-tiles per wave, FP32 keys
    1, 2 or 4; malformed lines are ignored.  Host-only, no GPU."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpkm.so not built")
    f = tmp_path / "tune.jsonl"
    f.write_text("\n".join([
        '{"s4": 104, "kt": 2, "kr": 1, "work": 1024, "u": 4, "fill": 1024}',   # ok
        '{"s4": 3, "kt": 1, "kr": 1, "work": 64, "u": 1, "fill": 512}',        # ok
        '{"s4": 3, "kt": 1, "kr": 1, "work": 128, "u": 2}',                    # ok (old format)
        '{"s4": 104, "kt": 2, "kr": 1, "work": 2048, "u": 1, "fill": 1024}',   # U=1 on FP16x3
        '{"s4": 3, "kt": 1, "kr": 1, "work": 64, "u": 3, "fill": 512}',        # U=3
        '{"s4": 3, "kt": 1, "kr": 1, "work": 64, "u": 2, "fill": 1000}',       # fill
        '{"s4": 12, "kt": 1, "kr": 0, "work": 64, "u": 2, "fill": 512}',       # s4 > 9
        '{"s4": 3, "kt": 1, "kr": 1, "work": 96, "u": 2, "fill": 512}',        # bucket not 2^p
        'garbage',
        '',
    ]))
    assert binding.pkm_tune_cache_load(f) == (3, 6)
    with pytest.raises(binding.PkmError):
        binding.pkm_tune_cache_load(None)


@pytest.mark.parametrize("n", [1, 2, 3, 10, 64, 200])
def test_host_eigensolver_matches_numpy(n):
    """pkm_sym_eig (the randomised-SVD setup's host eigensolver) against
    numpy's symmetric eigensolver: eigenvalues, orthonormal eigenvectors and
    the residual A Z - Z diag(w).  Host-only, no GPU."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpkm.so not built")
    rng = np.random.default_rng(100 + n)
    M = rng.standard_normal((n, n))
    for A in (M + M.T, M @ M.T, np.diag(rng.standard_normal(n))):
        w, Z = binding.pkm_sym_eig(A)
        scale = max(np.abs(A).max(), 1e-300)
        want = np.sort(np.linalg.eigvalsh(A))[::-1]
        assert np.all(np.diff(w) <= 0)
        assert np.allclose(w, want, rtol=0, atol=1e-12 * n * scale)
        assert np.allclose(Z.T @ Z, np.eye(n), atol=1e-12 * n)
        assert np.abs(A @ Z - Z * w).max() <= 1e-12 * n * scale


def test_host_eigensolver_degenerate_spectra():
    """Repeated eigenvalues (identity, a rank-1 matrix), the zero matrix and a
    tridiagonal input: still an orthonormal eigenbasis with the right
    eigenvalues.  Invalid input is rejected."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpkm.so not built")
    v = np.arange(1.0, 9.0)
    T = np.diag(np.full(8, 2.0)) - np.diag(np.ones(7), 1) - np.diag(np.ones(7), -1)
    for A, want in ((np.eye(8), np.ones(8)), (np.outer(v, v), np.r_[v @ v, np.zeros(7)]),
                    (np.zeros((5, 5)), np.zeros(5)),
                    (T, np.sort(2 - 2 * np.cos(np.arange(1, 9) * np.pi / 9))[::-1])):
        w, Z = binding.pkm_sym_eig(A)
        n = A.shape[0]
        assert np.allclose(w, want, atol=1e-12 * max(1.0, np.abs(A).max()) * n)
        assert np.allclose(Z.T @ Z, np.eye(n), atol=1e-12 * n)
        assert np.abs(A @ Z - Z * w).max() <= 1e-11 * max(1.0, np.abs(A).max())
    with pytest.raises(binding.PkmError):
        binding.pkm_sym_eig(np.array([[np.nan]]))
