"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and the host-only size query agrees with the oracle and
rejects invalid problems.  No GPU work is launched here."""
import os
import re

import pytest

from oracle import oracle as O
from paper_2103_14588_amd import inputs as IN

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "dirac_st.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dirac_st_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2103_14588_amd import dirac_st as D
    names = declared_functions()
    assert len(names) >= 7
    for n in names:
        assert hasattr(D._lib, n), n
    assert set(D.EXPORTS) <= set(names)


@pytest.mark.parametrize("spec", [
    IN.Spec(d=1, n=[64, 64]), IN.Spec(d=1, n=[1, 3]), IN.Spec(d=1, n=[2, 5]),
    IN.Spec(d=2, n=[7, 5, 3]), IN.Spec(d=2, n=[128, 128, 128]),
    IN.Spec(d=3, n=[12, 12, 12, 12]), IN.Spec(d=3, n=[32, 32, 32, 32]),
])
def test_sizes_match_oracle(spec):
    from paper_2103_14588_amd import dirac_st as D
    nrows, nnzb = D.sizes(spec)
    assert nrows == spec.nrows
    p = O.problem(spec.d, spec.n, spec.lens)
    assert nrows == O.nrows(p)
    if spec.nunknowns < 200000:
        assert nnzb == O.Matrix(p).export()[1].shape[0]
    # closed forms quoted for the large configurations
    if spec.n == [128, 128, 128]:
        assert (nrows, nnzb) == (2097152, 56328192)
    if spec.n == [32] * 4:
        assert (nrows, nnzb) == (1048576, 83165184)


@pytest.mark.parametrize("bad", [
    IN.Spec(d=4, n=[3, 3, 3, 3, 3]),
    IN.Spec(d=2, n=[3, 2, 5]),       # periodic axis shorter than 3
    IN.Spec(d=2, n=[0, 4, 4]),
    IN.Spec(d=1, n=[4, 4], lens=[1.0, -1.0]),
    IN.Spec(d=1, n=[4, 4], vkind=7),
])
def test_sizes_reject_invalid(bad):
    from paper_2103_14588_amd import dirac_st as D
    with pytest.raises(D.DiracError) as e:
        D.sizes(bad)
    assert e.value.code == D.EINVAL
    assert D.last_error()


def time_factors(nt, ht):
    """The 1D Galerkin time factors of the reduced operator written out entry
    by entry from the linear hat functions (mass and test-times-derivative
    integrals on [0, T] with the t = 0 node removed)."""
    import numpy as np
    M = np.zeros((nt, nt))
    Dm = np.zeros((nt, nt))
    for t in range(nt):
        M[t, t] = 2 * ht / 3 if t < nt - 1 else ht / 3
        if t > 0:
            M[t, t - 1], Dm[t, t - 1] = ht / 6, -0.5
        if t < nt - 1:
            M[t, t + 1], Dm[t, t + 1] = ht / 6, 0.5
    Dm[nt - 1, nt - 1] = 0.5
    return M, Dm


@pytest.mark.parametrize("nt,T", [(1, 1.0), (2, 1.0), (3, 0.7), (17, 1.0), (64, 2.0), (128, 1.0), (300, 1.0)])
def test_time_eigen_matches_library_eigensolver(nt, T):
    """Host part of the line preconditioner: eigenvalues of the time pencil
    against LAPACK's generalised eigensolver, eigenpair residuals, and
    W Q M = I (Q = W^{-1} M^{-1})."""
    import numpy as np
    import scipy.linalg as sl
    from paper_2103_14588_amd import dirac_st as D
    ht = T / nt
    lam, W, Q = D.time_eigen(nt, ht)
    M, Dm = time_factors(nt, ht)
    ref = sl.eig(Dm, M, right=False)
    scale = np.abs(ref).max()
    assert max(np.abs(ref - l).min() for l in lam) <= 1e-11 * scale
    assert max(np.abs(lam - r).min() for r in ref) <= 1e-11 * scale
    res = Dm @ W - (M @ W) * lam[None, :]
    assert np.abs(res).max() <= 1e-9 * (1 + scale * ht) * np.abs(W).max()
    assert np.abs(W @ Q @ M - np.eye(nt)).max() <= 1e-9


def test_time_eigen_rejects_bad_sizes():
    from paper_2103_14588_amd import dirac_st as D
    for nt, ht in ((0, 0.1), (2049, 1e-3), (4, -1.0)):
        with pytest.raises(D.DiracError):
            D.time_eigen(nt, ht)


def test_kernel_timers_host_side():
    """The timing switch and read-out are host-only: with nothing launched the
    counts are zero; an unknown kernel kind is rejected."""
    from paper_2103_14588_amd import dirac_st as D
    D.timing(True)
    for k in D.TIMED:
        assert D.timing_read(k) == (0, 0.0)
    D.timing(False)
    with pytest.raises(D.DiracError):
        D._check(D._lib.dirac_st_timing_read(99, D.C.byref(D._i64(0)), D.C.byref(D.C.c_double(0.0))))
