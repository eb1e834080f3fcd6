"""The heat-bath's rational approximation of x^{-1/2} (library host code, no GPU): its reported error is the
true maximum relative error on [lo, hi], the error equioscillates (2n + 1 sign changes between extrema of
equal size, the mark of the optimal approximation), poles and residues are positive, the error falls with
n, and the poles equal the Zolotarev points computed independently here with SciPy's Jacobi functions."""
import os

import numpy as np
import pytest

from paper_1710_09621_amd import eofa as E


def _lib_or_skip():
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("libeofa.so not built")


@pytest.mark.parametrize("lo,hi", [(0.45, 1.1), (0.4545, 2.178), (0.1, 10.0)])
def test_inv_sqrt_rational(lo, hi):
    _lib_or_skip()
    from scipy.special import ellipj, ellipk
    errs = []
    for n in range(1, 9):
        a0, a, b, err = E.inv_sqrt_rational(lo, hi, n)
        assert np.all(b > 0) and np.all(a > 0) and a0 > 0
        x = np.geomspace(lo, hi, 200001)
        r = a0 + sum(al / (x + bl) for al, bl in zip(a, b))
        e = np.sqrt(x) * r - 1
        errs.append(err)
        if err < 1e-13:  # rounding of the evaluation dominates below this
            continue
        assert abs(np.abs(e).max() - err) <= 1e-3 * err + 1e-15
        # extrema of alternating sign and equal size: at least 2n + 2 of them
        ext = np.r_[0, np.flatnonzero(np.diff(np.sign(np.diff(e))) != 0) + 1, len(e) - 1]
        big = ext[np.abs(e[ext]) > 0.99 * err]
        alternations = 1 + np.count_nonzero(np.diff(np.sign(e[big])) != 0)
        assert alternations >= 2 * n + 2, (n, alternations)
        # poles at -c_{2l-1}, c_j = lo sn^2 / cn^2 (j K' / (2n + 1)), k'^2 = 1 - lo / hi
        m = 1 - lo / hi
        sn, cn, _, _ = ellipj(np.arange(1, 2 * n + 1) * ellipk(m) / (2 * n + 1), m)
        c = lo * sn ** 2 / cn ** 2
        assert np.allclose(np.sort(b), np.sort(c[0::2]), rtol=1e-12)
    assert all(e2 < e1 or e2 < 1e-14 for e1, e2 in zip(errs, errs[1:]))
    if hi / lo < 6:  # the intervals the heat-bath uses by default: 6 poles reach 1e-9
        assert errs[5] < 1e-9


def test_inv_sqrt_rational_rejects_bad_interval():
    _lib_or_skip()
    for lo, hi, n in [(0.0, 1.0, 3), (1.0, 0.5, 3), (0.5, 1.0, 0), (0.5, 1.0, 9)]:
        with pytest.raises(E.EofaError):
            E.inv_sqrt_rational(lo, hi, n)
