"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host-side parameter selection follows the paper (Sec. 4.6)."""
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "se.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(se_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def se():
    import paper_2210_01255_amd as m
    return m


def test_library_exports_every_declared_symbol(se):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(se.lib, n), n
        assert n in se.EXPORTS, n


def test_version_and_status_strings(se):
    assert se.se_version() >= 100
    for code in se.STATUS:
        assert se.se_status_string(code)


def test_table4_xi_from_table3_nrc(se):
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "table4_xi.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 12
    for kernel, D, xi in rows:
        p = se.select_params(kernel=kernel, periodicity=int(D), tol=1e-8, tol_kind=se.TOL_ABS,
                             n_src=100000, source_q=1.0)
        assert abs(p["xi"] - float(xi)) < 5e-5, (kernel, D, p["xi"], xi)


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet", "stresslet"])
@pytest.mark.parametrize("D", [0, 1, 2, 3])
def test_parameter_rules(se, kernel, D):
    p = se.select_params(kernel=kernel, periodicity=D, tol=1e-8, tol_kind=se.TOL_ABS, n_src=100000,
                         source_q=1.0)
    P = p["P"]
    assert P % 2 == 0 and 4 <= P <= 32
    assert p["beta"] == 2.5 * P                       # eq. (PKB-parameters)
    assert p["nu_deg"] == min(P // 2 + 2, 10)
    for i in range(3):
        assert p["M"][i] % 4 == 0                       # multiples of f_M = 4
    # real-space estimate meets the tolerance at rc (step 1)
    assert p["est_real"] <= 1e-8 * (1 + 1e-9)
    # window estimate 10 U e^{-2.5 P} below tolerance after the pollution rule (steps 3-5)
    assert p["est_window"] <= 1e-8
    if D < 3:
        for i in range(D, 3):
            # free axes: window plus padding fit, delta L >= h P (Sec. 4.5)
            assert p["dL"][i] >= p["h"][i] * P - 1e-12
            assert abs(p["L_ext"][i] - p["h"][i] * p["M"][i]) < 1e-12
        R = p["R"]
        Lf = [p["L_ext"][i] for i in range(D, 3)]
        assert abs(R - math.sqrt(sum(v * v for v in Lf))) < 1e-12   # eq. (truncation-radius)
        assert p["s0"] >= 1 + R / min(Lf) - 1e-12                   # eq. (upsampling-factor-s0)


def test_metric_config_shape(se):
    p = se.select_params(kernel="stokeslet", periodicity=3, tol=1e-8, n_src=1_000_000, source_q=3e6)
    assert p["M"] == [240, 240, 240] and p["P"] == 14
    assert abs(p["xi"] - 86.41) < 0.05 and abs(p["rc"] - 0.0457) < 1e-4


def test_bad_arguments_are_rejected(se):
    with pytest.raises(se.SEError):
        se.select_params(kernel="stokeslet", periodicity=4, tol=1e-8, n_src=10)
    with pytest.raises(se.SEError):
        se.select_params(kernel="stokeslet", periodicity=3, tol=-1.0, n_src=10)
    with pytest.raises(se.SEError):
        se.select_params(kernel="stokeslet", periodicity=3, tol=1e-8, n_src=0)
    with pytest.raises(se.SEError):
        se.select_params(kernel="stokeslet", periodicity=3, tol=1e-8, n_src=10, box=(1.0, 0.0, 1.0))
    with pytest.raises(se.SEError):
        # window support above 32 points
        se.select_params(kernel="stokeslet", periodicity=3, tol=1e-30, tol_kind=se.TOL_ABS, n_src=10)


def test_pollution_rules(se):
    """Eq. (error-pollution-fix) and its alternative: P drops by 2, h by 1.05/1.1."""
    for D in (3, 2, 1):
        a = se.select_params(kernel="stokeslet", periodicity=D, tol=1e-8, n_src=10_000, safety=10)
        b = se.select_params(kernel="stokeslet", periodicity=D, tol=1e-8, n_src=10_000, safety=10,
                             pollution=se.POLLUTION_FINE)
        assert b["P"] == a["P"] - 2
        assert b["M"][0] >= a["M"][0]
    a = se.select_params(kernel="stokeslet", periodicity=0, tol=1e-8, n_src=10_000, safety=10)
    b = se.select_params(kernel="stokeslet", periodicity=0, tol=1e-8, n_src=10_000, safety=10,
                         pollution=se.POLLUTION_FINE)
    assert a["P"] == b["P"] and a["M"] == b["M"]  # D = 0 uses (h/1.1, P+2) either way
    with pytest.raises(se.SEError):
        se.select_params(kernel="stokeslet", periodicity=3, tol=1e-8, n_src=10, pollution=7)
