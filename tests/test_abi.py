"""The C-ABI library loads on the CPU, exports every symbol include/vp.h
declares, and its host-side reference data agrees with the oracle's
independently built tables (no device call is made here)."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import rules
from paper_2205_04401_amd import vp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vp_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(vp.EXPORTS)


C_TYPES = {"double": ctypes.c_double, "int": ctypes.c_int, "int32_t": ctypes.c_int32,
           "int64_t": ctypes.c_int64, "uint32_t": ctypes.c_uint32}


def header_struct(name):
    """(field, ctypes type) of a `typedef struct {...} name;` in vp.h, in order."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", src).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        fields += [(n.strip(), C_TYPES[ctype]) for n in names.split(",")]
    return fields


@pytest.mark.parametrize("cname, pyclass", [("vp_plan_opts", vp.PlanOpts), ("vp_plan_stats", vp.PlanStats),
                                            ("vp_far_config", vp.FarConfig)])
def test_struct_layouts_match_header(cname, pyclass):
    assert header_struct(cname) == list(pyclass._fields_)


def test_far_shape_names_match_header():
    src = open(HEADER).read()
    for name, value in vp.FAR_SHAPES.items():
        assert re.search(r"VP_FAR_" + name.upper() + r"\s*=\s*" + str(value) + r"\b", src), name


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(vp.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_fails_loudly_without_library(tmp_path):
    saved = vp._lib
    vp._lib = None
    try:
        with pytest.raises(vp.VPError):
            vp.load(str(tmp_path / "missing.so"))
    finally:
        vp._lib = saved


@pytest.mark.parametrize("p", range(1, 11))
def test_reference_nodes_match_oracle(p):
    assert np.abs(vp.ref_nodes(p) - rules.interp_nodes(p)).max() < 2e-15


@pytest.mark.parametrize("n", [2, 4, 8, 10, 16, 24])
def test_gauss_legendre_matches_oracle(n):
    x, _, w = vp.ref_rule(0, n)
    gx, gw = rules.gauss_legendre01(n)
    assert np.abs(x - gx).max() < 4e-16 and np.abs(w - gw).max() < 4e-15


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8])
def test_log_rule_matches_oracle(n):
    x, _, w = vp.ref_rule(1, n)
    gx, gw = rules.log_gauss01(n)
    assert np.abs(x - gx).max() < 4e-16 and np.abs(w - gw).max() < 4e-16


@pytest.mark.parametrize("q", [2, 3, 4, 7, 8, 12, 16, 20, 32])
def test_collapsed_rule_and_edge_weights_match_oracle(q):
    x, y, w = vp.ref_rule(2, q)
    X, W = rules.collapsed_gauss(q)
    assert np.abs(x - X[:, 0]).max() < 4e-16 and np.abs(y - X[:, 1]).max() < 4e-16
    assert np.abs(w - W).max() < 4e-16
    _, _, ew = vp.ref_rule(4, q)
    assert np.abs(ew - rules.edge_weights(q)).max() < 4e-16


@pytest.mark.parametrize("p", [1, 3, 4, 6, 8, 10])
def test_radial_rule_matches_oracle(p):
    r, a, b = vp.ref_rule(3, p)
    R, A, B = rules.radial_rule(p)
    assert np.abs(r - R).max() < 4e-16 and np.abs(a - A).max() < 4e-16 and np.abs(b - B).max() < 4e-16


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8, 10])
def test_folded_radial_rule(p):
    """The p + 1 node radial rule of the straight self pieces: exact for
    int_0^1 r^(m+1) dr = 1/(m+2) and int_0^1 r^(m+1) log r dr = -1/(m+2)^2,
    m <= p, and the same sum as the oracle's radial rule for polynomials of
    degree <= p and any log r0."""
    r, a, b = vp.ref_rule(5, p)
    assert len(r) == p + 1
    for m in range(p + 1):
        assert abs(np.sum(a * r ** m) - 1.0 / (m + 2)) < 1e-15
        assert abs(np.sum(b * r ** m) + 1.0 / (m + 2) ** 2) < 1e-15
    R, A, B = rules.radial_rule(p)
    rng = np.random.default_rng(p)
    for _ in range(5):
        c = rng.standard_normal(p + 1)
        lr0 = rng.uniform(-5.0, 1.0)
        phi = lambda x: np.polynomial.polynomial.polyval(x, c)
        folded = np.sum((a * lr0 + b) * phi(r))
        full = np.sum((A * lr0 + B) * phi(R))
        assert abs(folded - full) <= 1e-14 * max(1.0, abs(full))
    # a degree p + 1 term is not integrated exactly by the folded rule
    assert abs(np.sum(b * r ** (p + 1)) + 1.0 / (p + 3) ** 2) > 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_basis_connection_reproduces_koornwinder(p):
    """The row kernels' product basis (monic Legendre in 2x-1 times the
    homogeneous monic Legendre polynomial in the collapsed direction), through
    the library's connection table, gives the oracle's Koornwinder basis
    (Sec. 2.1) at points of the simplex, its vertices and edges included."""
    _, _, g = vp.ref_rule(6, p)
    n_p = rules.n_basis(p)
    g = np.asarray(g).reshape(n_p, p + 1)
    rng = np.random.default_rng(60 + p)
    u, v = rng.random(200), rng.random(200)
    flip = u + v > 1.0
    u[flip], v[flip] = 1.0 - u[flip], 1.0 - v[flip]
    x = np.concatenate([u, [0.0, 1.0, 0.0, 0.5, 0.0, 0.5, 1.0 / 3.0]])
    y = np.concatenate([v, [0.0, 0.0, 1.0, 0.0, 0.5, 0.5, 1.0 / 3.0]])
    t, z = 1.0 - x, 2.0 * x - 1.0
    s = 2.0 * y - t
    pm = [np.ones_like(z), z]
    qm = [np.ones_like(z), s]
    for j in range(1, p):
        e = j * j / (4.0 * j * j - 1.0)
        pm.append(z * pm[j] - e * pm[j - 1])
        qm.append(s * qm[j] - e * t * t * qm[j - 1])
    got = np.zeros((len(x), n_p))
    for n in range(p + 1):
        for m in range(n + 1):
            i = n * (n + 1) // 2 + m
            assert np.all(g[i, n - m + 1:] == 0.0)
            got[:, i] = sum(g[i, j] * qm[m] * pm[j] for j in range(n - m + 1))
    ref = rules.koornwinder(p, x, y)
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    with pytest.raises(vp.VPError):
        vp.ref_rule(6, 7)


def test_invalid_rule_requests_are_rejected():
    with pytest.raises(vp.VPError) as e:
        vp.ref_rule(7, 4)
    assert e.value.status == vp.VP_EINVAL
    with pytest.raises(vp.VPError):
        vp.ref_nodes(0)
    with pytest.raises(vp.VPError):
        vp.ref_nodes(11)
