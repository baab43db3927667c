"""Host-side checks of libxyz that need no GPU: the shared library loads,
exports every function include/xyz.h declares, and its host logic (the
integer threshold of eq. (1)) agrees with the definition."""
import os
import re

import numpy as np
import pytest

import paper_1610_05108_amd as xyz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "xyz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xyz_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = xyz.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(xyz.EXPORTS)


def test_version_string():
    assert "gfx950" in xyz.xyz_version()


@pytest.mark.parametrize("n", [1, 2, 7, 200, 859, 2000, 5000])
def test_smin_matches_strict_threshold(n):
    """eq. (1) keeps s/n > kappa with s/n the binary64 quotient; the library's
    integer threshold must select exactly those s."""
    kappas = [-1.5, -1.0, -0.3, -1e-9, 0.0, 1e-12, 0.05, 0.1, 0.12, 0.3, 1 / 3, 0.5, 0.999, 1.0, 2.0]
    kappas += [s / n for s in range(-n, n + 1, max(1, n // 17))]
    s = np.arange(-n, n + 1)
    for kappa in kappas:
        smin = xyz.xyz_smin(n, kappa, False)
        keep = np.array([(int(v) / n) > kappa for v in s])
        assert np.array_equal(keep, s >= smin), (n, kappa, smin)
        smin2 = xyz.xyz_smin(n, kappa, True)
        keep2 = np.array([(abs(int(v)) / n) > kappa for v in s])
        assert np.array_equal(keep2, np.abs(s) >= smin2), (n, kappa, smin2)


def test_init_without_gpu_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(xyz.XyzError):
        xyz.xyz_init(0)
