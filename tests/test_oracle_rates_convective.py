"""Pins of the oracle's convective fluxes and of its reaction-rate law.

Convective terms (Section 2.1, eq. cns): the oracle's convective-only
right-hand side must converge at eighth order to minus the spectral
divergence of (rho u, rho u u + p I, (rho E + p) u, rho Y_k u) on smooth
periodic fields in which every primitive (p included) varies.

Rate law (the readings restated in the oracle: reversible Arrhenius
reactions, equilibrium constants from the NASA-7 Gibbs functions):
  * thermodynamic equilibrium: with concentrations c_k = (p_ref/(R T))
    exp(-g_k/(R T) + sum_e lambda_e n_ek) every element-balanced reaction has
    sum_k nu_k mu_k = 0 for any element potentials lambda_e, so every rate of
    progress must vanish (the Gibbs functions are evaluated here from the
    NASA-7 definition, not by the oracle);
  * van 't Hoff: d ln K_p / dT = Delta h / (R T^2), with Delta h from the
    species enthalpies, and K_p = K_c (R T / p_ref)^{Delta nu} taken from the
    oracle's forward and reverse rate constants;
  * Arrhenius slope: d ln k_f / d ln T = b + E_a / (R T);
  * mass action: with the products absent, scaling every concentration by
    s at fixed temperature scales the rate of progress by s^(forward order).
"""
import numpy as np
import pytest

from synth import mechanism

RU = 8.31446261815324
PREF = 101325.0


@pytest.fixture(scope="module")
def mechs(orc):
    return {k: orc.Mechanism(mechanism.load(k)) for k in ("mech9", "mech9le", "mech21")}


# ----------------------------------------------------------- NASA-7 (test side)
def nasa_h_RT(a, T):
    return a[0] + a[1] * T / 2 + a[2] * T ** 2 / 3 + a[3] * T ** 3 / 4 + a[4] * T ** 4 / 5 + a[5] / T


def nasa_s_R(a, T):
    return a[0] * np.log(T) + a[1] * T + a[2] * T ** 2 / 2 + a[3] * T ** 3 / 3 + a[4] * T ** 4 / 4 + a[6]


def gibbs_RT(m, T):
    return np.array([nasa_h_RT(a, T) - nasa_s_R(a, T) for a in m["nasa"]])


def one_reaction(m, j):
    one = dict(m)
    for key in ("A", "b", "Ea", "nu_f", "nu_r"):
        one[key] = np.asarray(m[key])[j:j + 1]
    one["nr"] = 1
    return one


def state_from_concentrations(orc, om, T, c):
    """Conserved state of one cell at rest with temperature T and molar
    concentrations c (mol/m^3)."""
    W = om.mech["W"]
    rho = np.sum(c * W)
    Y = c * W / rho
    p = RU * T * np.sum(c)
    prim = dict(p=np.array([p]), T=np.array([T]), Y=Y[:, None], u=np.zeros((3, 1)))
    return orc.prim_to_cons(om, prim)


# ------------------------------------------------------------------ equilibrium
@pytest.mark.parametrize("key", ["mech9", "mech21"])
def test_every_reaction_vanishes_at_thermodynamic_equilibrium(orc, mechs, key):
    om = mechs[key]
    m = om.mech
    comp = np.asarray(m["composition"], dtype=float)         # [ns][elements]
    rng = np.random.default_rng(11)
    W = m["W"]
    nuf = np.asarray(m["nu_f"])
    nur = np.asarray(m["nu_r"])
    for T in (700.0, 1400.0, 2300.0):
        for trial in range(2):
            base = np.log(PREF / (RU * T)) - gibbs_RT(m, T)
            # element potentials: a least-squares choice that brings every
            # concentration near p_ref/(R T), plus a random offset (any
            # lambda gives an equilibrium state)
            lam, *_ = np.linalg.lstsq(comp, np.log(PREF / (RU * T)) - 1.0 - base, rcond=None)
            lam += rng.uniform(-1.0, 1.0, comp.shape[1])
            c = np.exp(base + comp @ lam)
            U = state_from_concentrations(orc, om, T, c)
            for j in range(om.nr):
                oj = orc.Mechanism(one_reaction(m, j))
                w = orc.production(oj, U)[:, 0]
                k = int(np.argmax(np.abs(nur[j] - nuf[j])))
                q = w[k] / (W[k] * (nur[j, k] - nuf[j, k]))
                kf, _ = orc.rate_constants(oj, T)
                fwd = kf[0] * np.prod(c ** nuf[j])
                assert abs(q) <= 1e-9 * fwd, (key, T, j, q / fwd)


def test_disequilibrium_is_detected(orc, mechs):
    # the same construction with one species displaced gives non-zero rates
    om = mechs["mech9"]
    m = om.mech
    T = 1400.0
    comp = np.asarray(m["composition"], dtype=float)
    base = np.log(PREF / (RU * T)) - gibbs_RT(m, T)
    lam, *_ = np.linalg.lstsq(comp, np.log(PREF / (RU * T)) - 1.0 - base, rcond=None)
    c = np.exp(base + comp @ lam)
    c[2] *= 3.0
    U = state_from_concentrations(orc, om, T, c)
    w = orc.production(om, U)[:, 0]
    assert np.abs(w).max() > 0
    nuf = np.asarray(m["nu_f"])
    nur = np.asarray(m["nu_r"])
    touched = [j for j in range(om.nr) if nuf[j, 2] or nur[j, 2]]
    assert touched
    for j in touched:
        oj = orc.Mechanism(one_reaction(m, j))
        wj = orc.production(oj, U)[:, 0]
        kf, _ = orc.rate_constants(oj, T)
        assert np.abs(wj).max() > 1e-3 * kf[0] * np.prod(c ** nuf[j]) * m["W"].min()


# ------------------------------------------------------------------ van 't Hoff
@pytest.mark.parametrize("key", ["mech9", "mech21"])
def test_van_t_hoff(orc, mechs, key):
    om = mechs[key]
    m = om.mech
    dnu = (np.asarray(m["nu_r"]) - np.asarray(m["nu_f"])).astype(float)
    dnu_tot = dnu.sum(axis=1)

    def lnKp(T):
        kf, kr = orc.rate_constants(om, T)
        return np.log(kf / kr) + dnu_tot * np.log(RU * T / PREF)

    for T in (500.0, 1200.0, 2500.0):
        h = 1e-4 * T
        fd = (lnKp(T + h) - lnKp(T - h)) / (2 * h)
        # Delta h / (R T^2) from the species enthalpies h_k = R T (h/RT)_k
        dh_RT = dnu @ np.array([nasa_h_RT(a, T) for a in m["nasa"]])
        expect = dh_RT / T
        np.testing.assert_allclose(fd, expect, rtol=1e-6, atol=1e-7 * np.abs(expect).max())


# ------------------------------------------------------------------ Arrhenius
@pytest.mark.parametrize("key", ["mech9", "mech21"])
def test_arrhenius_slope(orc, mechs, key):
    om = mechs[key]
    m = om.mech
    for T in (400.0, 1000.0, 2600.0):
        eps = 1e-4
        kp, _ = orc.rate_constants(om, T * np.exp(eps))
        km, _ = orc.rate_constants(om, T * np.exp(-eps))
        slope = (np.log(kp) - np.log(km)) / (2 * eps)
        expect = np.asarray(m["b"]) + np.asarray(m["Ea"]) / (RU * T)
        np.testing.assert_allclose(slope, expect, rtol=1e-6, atol=1e-7)
    # the prefactor scales k_f linearly and leaves the equilibrium constant
    m2 = dict(m)
    m2["A"] = np.asarray(m["A"]) * 3.0
    kf1, kr1 = orc.rate_constants(om, 1300.0)
    kf3, kr3 = orc.rate_constants(orc.Mechanism(m2), 1300.0)
    np.testing.assert_allclose(kf3, 3.0 * kf1, rtol=1e-14)
    np.testing.assert_allclose(kf3 / kr3, kf1 / kr1, rtol=1e-14)


def test_production_follows_the_arrhenius_slope(orc, mechs):
    # with the products absent the rate of progress is k_f(T) prod c^nu' at
    # fixed concentrations, so d ln q / d ln T = b + E_a / (R T) through the
    # production routine itself
    om = mechs["mech21"]
    m = om.mech
    nuf = np.asarray(m["nu_f"])
    nur = np.asarray(m["nu_r"])
    rng = np.random.default_rng(6)
    for j in range(0, om.nr, 5):
        oj = orc.Mechanism(one_reaction(m, j))
        c = rng.uniform(1.0, 5.0, om.ns)
        c[nur[j] > 0] = 0.0
        k = int(np.argmax(nuf[j]))
        for T in (600.0, 1800.0):
            eps = 1e-4
            lq = []
            for TT in (T * np.exp(eps), T * np.exp(-eps)):
                U = state_from_concentrations(orc, om, TT, c)
                w = orc.production(oj, U)[:, 0]
                lq.append(np.log(w[k] / (m["W"][k] * (nur[j, k] - nuf[j, k]))))
            slope = (lq[0] - lq[1]) / (2 * eps)
            assert slope == pytest.approx(m["b"][j] + m["Ea"][j] / (RU * T), rel=1e-6, abs=1e-6), (j, T)


# ------------------------------------------------------------------ mass action
def test_mass_action_order(orc, mechs):
    om = mechs["mech21"]
    m = om.mech
    nuf = np.asarray(m["nu_f"])
    nur = np.asarray(m["nu_r"])
    rng = np.random.default_rng(5)
    T = 1500.0
    for j in range(0, om.nr, 7):
        oj = orc.Mechanism(one_reaction(m, j))
        c = rng.uniform(1.0, 5.0, om.ns)
        c[nur[j] > 0] = 0.0                     # products absent: no reverse term
        k = int(np.argmax(nuf[j]))
        order = nuf[j].sum()
        q = []
        for s in (1.0, 2.0):
            U = state_from_concentrations(orc, om, T, s * c)
            w = orc.production(oj, U)[:, 0]
            q.append(w[k] / (m["W"][k] * (nur[j, k] - nuf[j, k])))
        assert q[0] > 0
        assert q[1] / q[0] == pytest.approx(2.0 ** order, rel=1e-10), (j, order)


# ------------------------------------------------------------ convective terms
def _sd(f, axis, dx):
    n = f.shape[axis]
    k = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    shape = [1] * f.ndim
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def _div(F, dx):
    # axes of a [z][y][x] field: x = 2, y = 1, z = 0
    return _sd(F[0], 2, dx) + _sd(F[1], 1, dx) + _sd(F[2], 0, dx)


def _flow(n, ns):
    dx = 1e-4
    L = n * dx
    z, y, x = np.meshgrid(*(np.arange(n) * dx,) * 3, indexing="ij")
    k = 2 * np.pi / L
    u = np.stack([30 * np.sin(k * y) + 20 * np.cos(k * (x + z)),
                  -20 * np.cos(k * z) + 10 * np.sin(2 * k * x),
                  10 * np.sin(k * (x - y)) + 15 * np.cos(k * y)])
    T = 1000 + 300 * np.sin(k * x) * np.cos(k * y) + 100 * np.cos(k * z)
    p = 101325.0 * (1 + 0.2 * np.cos(k * (x + y)) + 0.1 * np.sin(k * z))
    Ya = np.random.default_rng(7).dirichlet(np.ones(ns))
    Yb = np.random.default_rng(8).dirichlet(np.ones(ns))
    w = 0.5 * (1 + np.sin(k * (y + z)))
    Y = w * Ya[:, None, None, None] + (1 - w) * Yb[:, None, None, None]
    return dict(p=p, T=T, Y=Y, u=u), dx


@pytest.mark.parametrize("key", ["mech9", "mech21"])
def test_convective_terms_converge_to_spectral_flux_divergence(orc, mechs, key):
    om = mechs[key]
    errs = []
    for n in (32, 64):
        prim, dx = _flow(n, om.ns)
        U = orc.prim_to_cons(om, prim)
        f = orc.rhs(om, U, dx, parts=orc.HYP)
        u, p = prim["u"], prim["p"]
        rho, rhoE = U[0], U[4]
        ref = [-_div([rho * u[d] for d in range(3)], dx)]
        for i in range(3):
            ref.append(-_div([rho * u[i] * u[d] + (p if i == d else 0.0) for d in range(3)], dx))
        ref.append(-_div([(rhoE + p) * u[d] for d in range(3)], dx))
        for kk in range(om.ns):
            ref.append(-_div([U[5 + kk] * u[d] for d in range(3)], dx))
        e = [np.abs(f[q] - ref[q]).max() / np.abs(ref[q]).max() for q in range(U.shape[0])]
        errs.append(max(e))
    assert errs[-1] < 2e-7, errs
    assert np.log2(errs[0] / errs[1]) > 7.0, errs
