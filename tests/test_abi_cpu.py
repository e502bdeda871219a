"""CPU-side checks of the C ABI: the library loads and exports every symbol the
header declares, and the header and binding agree on names and constants."""
import ctypes
import os
import re
import subprocess

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
