"""Pins of the oracle's multiresolution operators and fluxes (CPU only).

Projection / prediction: Sec. 2 "Projection and prediction operators"
(projection = children mean; 1D prediction q -/+ (q_{i+1}-q_{i-1})/8; the
operator must be local and satisfy projection o prediction = identity;
degree-2 interpolation on cell averages).
"""
from fractions import Fraction as Fr
import itertools
import math

import numpy as np
import pytest

from paper_1905_08717_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _stencil_index(o):
    ox, oy, oz = (list(o) + [0, 0])[:3]
    return (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)


def _exact_avg_poly(coef, lo, h):
    """Exact average of prod_a p_a(x_a) over the box [lo, lo+h]^d, p_a given
    by polynomial coefficients (ascending) as Fractions."""
    val = Fr(1)
    for a, c in enumerate(coef):
        # average of sum_j c_j x^j over [l, l+h]
        l = lo[a]
        s = Fr(0)
        for j, cj in enumerate(c):
            s += cj * ((l + h) ** (j + 1) - l ** (j + 1)) / (j + 1)
        val *= s / h
    return val


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_prediction_exact_on_per_dimension_quadratics(oracle_mod, dim):
    # degree-2 interpolation on cell averages (Harten) is exact for quadratics;
    # in multi-D the tensor product is exact for products of quadratics.
    rng = np.random.default_rng(1 + dim)
    for trial in range(5):
        coef = [[Fr(int(v), 8) for v in rng.integers(-8, 9, 3)] for _ in range(dim)]
        h = Fr(1, 4)
        center = [Fr(int(v)) * h for v in rng.integers(-3, 4, dim)]
        st = np.zeros(27)
        for o in itertools.product([-1, 0, 1], repeat=dim):
            lo = [center[a] + o[a] * h for a in range(dim)]
            st[_stencil_index(o)] = float(_exact_avg_poly(coef, lo, h))
        ch = oracle_mod.predict(dim, st[None, :])
        for cb in range(1 << dim):
            bits = [(cb >> a) & 1 for a in range(dim)]
            lo = [center[a] + bits[a] * h / 2 for a in range(dim)]
            exact = float(_exact_avg_poly(coef, lo, h / 2))
            assert ch[cb, 0] == pytest.approx(exact, rel=1e-14, abs=1e-15), (dim, trial, cb)


def test_prediction_1d_matches_printed_formula(oracle_mod):
    # Sec. 2: child 2i = q_i - (q_{i+1} - q_{i-1})/8, child 2i+1 = q_i + (...)/8
    st = np.zeros(27)
    st[_stencil_index([-1])], st[_stencil_index([0])], st[_stencil_index([1])] = 3.0, 5.0, 11.0
    ch = oracle_mod.predict(1, st[None, :])
    assert ch[0, 0] == 5.0 - (11.0 - 3.0) / 8
    assert ch[1, 0] == 5.0 + (11.0 - 3.0) / 8


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_projection_of_prediction_is_identity(oracle_mod, dim):
    # consistency P_{l+1->l} o P_{l->l+1} = Id, exact on dyadic data
    rng = np.random.default_rng(7)
    for _ in range(20):
        st = np.zeros((2, 27))
        for o in itertools.product([-1, 0, 1], repeat=dim):
            st[:, _stencil_index(o)] = rng.integers(-1000, 1000, 2) / 16.0
        ch = oracle_mod.predict(dim, st)
        par = oracle_mod.project(dim, ch)
        assert np.array_equal(par, st[:, _stencil_index([0] * dim)])


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_prediction_is_local_and_linear(oracle_mod, dim):
    # locality: only the parent and its nearest neighbours enter (3^d cells)
    rng = np.random.default_rng(3)
    base = rng.normal(size=(1, 27))
    ch0 = oracle_mod.predict(dim, base)
    for o in itertools.product([-1, 0, 1], repeat=3):
        if any(o[a] != 0 for a in range(dim, 3)):
            pert = base.copy()
            pert[0, _stencil_index(o)] += 1.0
            assert np.array_equal(oracle_mod.predict(dim, pert), ch0)


def test_projection_is_children_mean(oracle_mod):
    ch = np.array([[1.0], [2.0], [4.0], [9.0]])
    assert oracle_mod.project(2, ch)[0] == 4.0
    ch3 = np.arange(8.0)[:, None]
    assert oracle_mod.project(3, ch3)[0] == 3.5


def _mk(oracle_mod, cfg):
    return oracle_mod.Oracle(cfg)


def test_mr_transform_round_trip_exact_without_threshold(oracle_mod):
    # MR transform q^L <-> (D^L..D^1, q^0) is invertible (Sec. 2): with eps=0
    # the full tree is kept and reconstruction returns the input exactly.
    for cfg in (W.burgers_1d(L=8, eps=0.0), W.nagumo_2d(L=6, eps=0.0)):
        o = _mk(oracle_mod, cfg)
        q = W.initial_data(cfg)
        o.load_finest(q)
        assert np.array_equal(o.reconstruct(), q)


def test_thresholded_reconstruction_error_bounded_by_eps(oracle_mod):
    # details below eps are dropped: the reconstruction error is O(eps)
    for eps in (1e-2, 1e-3, 1e-4):
        cfg = W.nagumo_2d(L=7, eps=eps)
        o = _mk(oracle_mod, cfg)
        q = W.initial_data(cfg)
        o.load_finest(q)
        err = np.abs(o.reconstruct() - q)
        assert err.max() <= 4 * eps, (eps, err.max())
        st = o.stats()
        assert sum(st["leaves"]) < q.shape[1]


def test_details_vanish_on_quadratics(oracle_mod):
    # details = q - q~ vanish where the prediction is exact (Sec. 2)
    cfg = dict(dim=1, L=7, l0=2, eps=0.0, pde="burgers", nu=0.0, bc="neumann")
    o = _mk(oracle_mod, cfg)
    n = 1 << 7
    xe = np.arange(n + 1) / n
    prim = xe ** 3 / 3.0 - 0.5 * xe ** 2          # antiderivative of x^2 - x
    q = ((prim[1:] - prim[:-1]) * n)[None, :]
    o.load_finest(q)
    for lev in range(3, 7):
        D = o.details(lev)
        nn = 1 << lev
        interior = D[2:nn - 2]
        assert np.all(interior >= 0) and interior.max() < 1e-14


# ---------------------------------------------------------------------------
# fluxes


def _cfg_flux(pde, dim=1, **kw):
    c = dict(dim=dim, L=6, l0=2, eps=0.0, pde=pde, nu=kw.pop("nu", 0.0), bc="periodic")
    c.update(kw)
    return c


def test_godunov_burgers_flux_cases(oracle_mod):
    o = _mk(oracle_mod, _cfg_flux("burgers", recon=0))
    f = lambda l, r: o.face_flux(3, 0, np.array([[l], [l], [r], [r]]))[0]
    assert f(2.0, 1.0) == 2.0          # right-moving shock: f(uL)
    assert f(-1.0, -2.0) == 2.0        # left-moving shock: f(uR)
    assert f(-1.0, 1.0) == 0.0         # transonic rarefaction: f(0)
    assert f(1.0, -3.0) == 4.5         # shock with negative speed: f(uR)
    assert f(3.0, -1.0) == 4.5         # shock with positive speed: f(uL)


def test_muscl_minmod_limits_at_extrema(oracle_mod):
    o = _mk(oracle_mod, _cfg_flux("advection", recon=1, adv_vel=[1.0, 0, 0]))
    # monotone data: qL = q_a + minmod slope / 2
    F = o.face_flux(3, 0, np.array([[0.0], [1.0], [3.0], [4.0]]))
    assert F[0] == 1.0 + 0.5 * 1.0
    # extremum at a: slope 0 -> first order
    F = o.face_flux(3, 0, np.array([[2.0], [3.0], [1.0], [0.0]]))
    assert F[0] == 3.0


def _euler_phys_flux(d, q, ax, gamma=1.4):
    rho = q[0]
    u = q[1:1 + d] / rho
    E = q[d + 1]
    p = (gamma - 1) * (E - 0.5 * rho * np.dot(u, u))
    F = np.zeros(d + 2)
    F[0] = rho * u[ax]
    F[1:1 + d] = rho * u[ax] * u
    F[1 + ax] += p
    F[d + 1] = (E + p) * u[ax]
    return F


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_ausm_plus_consistent_with_physical_flux(oracle_mod, dim):
    # F(q, q) = f(q): consistency of the AUSM+ flux (Liou 1996)
    o = _mk(oracle_mod, _cfg_flux("euler", dim=dim, recon=1, gamma=1.4))
    rng = np.random.default_rng(11)
    for _ in range(50):
        rho, p = rng.uniform(0.1, 3.0, 2)
        u = rng.uniform(-2.5, 2.5, dim)
        q = np.array(W.euler_state(rho, *(list(u) + [0, 0])[:3], p, 1.4, dim))
        for ax in range(dim):
            F = o.face_flux(3, ax, np.tile(q, (4, 1)))
            assert np.allclose(F, _euler_phys_flux(dim, q, ax), rtol=1e-13, atol=1e-13)


def test_ausm_plus_supersonic_upwinding(oracle_mod):
    # |M| >= 1 on both sides: the flux is the physical flux of the upwind side
    o = _mk(oracle_mod, _cfg_flux("euler", dim=1, recon=0, gamma=1.4))
    qL = np.array(W.euler_state(1.0, 3.0, 0, 0, 1.0, 1.4, 1))
    qR = np.array(W.euler_state(0.5, 2.9, 0, 0, 0.8, 1.4, 1))
    F = o.face_flux(3, 0, np.array([qL, qL, qR, qR]))
    assert np.allclose(F, _euler_phys_flux(1, qL, 0), rtol=1e-14)
    F = o.face_flux(3, 0, np.array([qR * [1, -1, 1], qR * [1, -1, 1], qL * [1, -1, 1], qL * [1, -1, 1]]))
    assert np.allclose(F, _euler_phys_flux(1, qL * [1, -1, 1], 0), rtol=1e-14)


def test_ausm_plus_splitting_polynomials(oracle_mod):
    # M+(M) + M-(M) = M and P+(M) + P-(M) = 1 for every M: with equal states
    # the mass flux is rho*u exactly and the pressure term is p.
    o = _mk(oracle_mod, _cfg_flux("euler", dim=1, recon=0, gamma=1.4))
    for M in np.linspace(-1.5, 1.5, 31):
        rho, p = 1.3, 0.7
        a = math.sqrt(1.4 * p / rho)
        q = np.array(W.euler_state(rho, M * a, 0, 0, p, 1.4, 1))
        F = o.face_flux(3, 0, np.tile(q, (4, 1)))
        assert F[0] == pytest.approx(rho * M * a, rel=1e-13, abs=1e-14)
        assert F[1] == pytest.approx(rho * (M * a) ** 2 + p, rel=1e-13)
