"""Pins of the oracle's thermochemistry and right-hand side against
identities, invariants and a spectral evaluation of the continuous operators
(Section 2.1 and the readings restated in the oracle)."""
import numpy as np
import pytest

from synth import fields, mechanism

RU = 8.31446261815324


@pytest.fixture(scope="module")
def mechs(orc):
    return {k: orc.Mechanism(mechanism.load(k)) for k in ("mech9", "mech9le", "mech12", "mech21")}


def _state(orc, om, shape=(8, 8, 8), seed=3):
    prim = fields.sines(shape, 1e-4, om.ns, seed)
    return prim, orc.prim_to_cons(om, prim)


def test_nasa_polynomials_are_consistent(orc, mechs):
    # d(h/R)/dT = c_p/R and d(s/R)/dT = (c_p/R)/T
    om = mechs["mech21"]
    for T in (300.0, 1000.0, 2500.0):
        h = 1e-3
        cp, hRT, sR = orc.species_thermo(om, T)
        _, hp, sp_ = orc.species_thermo(om, T + h)
        _, hm, sm = orc.species_thermo(om, T - h)
        np.testing.assert_allclose(((T + h) * hp - (T - h) * hm) / (2 * h), cp, rtol=1e-9)
        np.testing.assert_allclose((sp_ - sm) / (2 * h), cp / T, rtol=1e-8)
        assert np.all((cp >= 2.5 - 1e-12) & (cp <= 7.0 + 1e-12))


def test_temperature_round_trip_and_eos(orc, mechs):
    for om in mechs.values():
        prim, U = _state(orc, om)
        out = orc.cons_to_prim(om, U)
        np.testing.assert_allclose(out[4], prim["T"], rtol=1e-13)
        np.testing.assert_allclose(out[5], prim["p"], rtol=1e-13)
        np.testing.assert_allclose(out[1:4], prim["u"], rtol=1e-13, atol=1e-13)


def test_internal_energy_derivative_is_cv(orc, mechs):
    # e(T) from the conversion: (e(T+h) - e(T-h)) / 2h equals c_v = c_p - R/W
    om = mechs["mech9"]
    m = om.mech
    Y = np.random.default_rng(0).dirichlet(np.ones(om.ns))
    for T in (400.0, 1500.0):
        def e_of(TT):
            prim = dict(p=np.array([1e5]), T=np.array([TT]), Y=Y[:, None], u=np.zeros((3, 1)))
            U = orc.prim_to_cons(om, prim)
            return U[4, 0] / U[0, 0]
        h = 1e-2
        cv_fd = (e_of(T + h) - e_of(T - h)) / (2 * h)
        cp, _, _ = orc.species_thermo(om, T)
        cv = np.sum(Y * RU / m["W"] * (cp - 1.0))
        assert cv_fd == pytest.approx(cv, rel=1e-7)


def test_production_conserves_mass_and_elements(orc, mechs):
    for om in mechs.values():
        m = om.mech
        prim, U = _state(orc, om)
        w = orc.production(om, U).reshape(om.ns, -1)
        scale = np.abs(w).sum(axis=0) + 1e-300
        assert np.abs(w.sum(axis=0) / scale).max() < 1e-13
        comp = m["composition"]                     # [ns][elements]
        moles = w / m["W"][:, None]
        el = comp.T @ moles
        escale = np.abs(comp).T @ np.abs(moles) + 1e-300
        assert np.abs(el / escale).max() < 1e-13


def test_lnA_derivative_is_single_reaction_rate(orc, mechs):
    # d(rho omega_k)/d lnA_j = W_k nu_kj q_j, the production of reaction j alone
    om = mechs["mech9"]
    m = om.mech
    prim, U = _state(orc, om, shape=(4, 4, 4))
    for j in (0, 7, 20):
        wA = np.zeros(om.nr)
        wA[j] = 1.0
        _, jvp = orc.rhs_jvp(om, U, 1e-4, np.zeros_like(U), wA, parts=orc.REACT)
        one = dict(m)
        for key in ("A", "b", "Ea", "nu_f", "nu_r"):
            one[key] = m[key][j:j + 1]
        one["nr"] = 1
        w = orc.production(orc.Mechanism(one), U)
        np.testing.assert_allclose(jvp[5:], w, rtol=1e-12, atol=1e-12 * np.abs(w).max())
        assert np.abs(jvp[:5]).max() == 0.0


def test_jvp_matches_central_differences(orc, mechs):
    om = mechs["mech9le"]
    prim, U = _state(orc, om, shape=(6, 5, 4))
    rng = np.random.default_rng(1)
    w = rng.standard_normal(U.shape) * np.sqrt(np.mean(U ** 2, axis=(1, 2, 3), keepdims=True))
    wA = rng.standard_normal(om.nr)
    _, jvp = orc.rhs_jvp(om, U, 1e-4, w, wA)
    eps = 1e-6
    m = om.mech
    mp, mm = dict(m), dict(m)
    mp["A"] = m["A"] * np.exp(eps * wA)
    mm["A"] = m["A"] * np.exp(-eps * wA)
    fp = orc.rhs(orc.Mechanism(mp), U + eps * w, 1e-4)
    fm = orc.rhs(orc.Mechanism(mm), U - eps * w, 1e-4)
    fd = (fp - fm) / (2 * eps)
    for q in range(U.shape[0]):
        scale = np.abs(jvp[q]).max()
        assert np.abs(fd[q] - jvp[q]).max() <= 2e-6 * scale, q


def test_uniform_state_at_rest_is_a_0d_reactor(orc, mechs):
    om = mechs["mech9"]
    Y = np.random.default_rng(2).dirichlet(np.ones(om.ns))
    shape = (8, 8, 8)
    prim = dict(p=np.full(shape, 101325.0), T=np.full(shape, 1200.0),
                Y=np.broadcast_to(Y[:, None, None, None], (om.ns,) + shape).copy(),
                u=np.zeros((3,) + shape))
    U = orc.prim_to_cons(om, prim)
    ad = orc.rhs(om, U, 1e-4, parts=orc.AD)
    # differences of equal samples: the convective and first-derivative terms
    # vanish exactly; the narrow rows sum to zero only up to rounding
    conv = orc.rhs(om, U, 1e-4, parts=orc.HYP)
    assert np.abs(conv).max() == 0.0
    scale = np.abs(U).max(axis=(1, 2, 3)) / 1e-8
    assert np.all(np.abs(ad).max(axis=(1, 2, 3)) <= 1e-12 * scale)
    full = orc.rhs(om, U, 1e-4, parts=orc.REACT)
    w = orc.production(om, U)
    np.testing.assert_array_equal(full[5:], w)
    assert np.abs(full[:5]).max() == 0.0


def test_species_sum_equals_continuity(orc, mechs):
    for key in ("mech9", "mech9le"):
        om = mechs[key]
        prim, U = _state(orc, om)
        U[5:] *= U[0] / U[5:].sum(axis=0)      # sum_k rho Y_k = rho to rounding
        f = orc.rhs(om, U, 1e-4)
        scale = np.abs(f[5:]).max()
        assert np.abs(f[5:].sum(axis=0) - f[0]).max() <= 1e-12 * scale


def test_periodic_box_conserves_mass_momentum_energy(orc, mechs):
    om = mechs["mech9"]          # unity Lewis numbers: the correction velocity vanishes
    prim, U = _state(orc, om)
    f = orc.rhs(om, U, 1e-4, parts=orc.AD)
    for q in range(5):
        assert abs(f[q].sum()) <= 1e-12 * np.abs(f[q]).sum(), q
    for q in range(5, U.shape[0]):   # species: flux form up to the V_c terms
        assert abs(f[q].sum()) <= 1e-10 * np.abs(f[q]).sum(), q


def test_translation_and_axis_permutation_equivariance(orc, mechs):
    om = mechs["mech9le"]
    prim, U = _state(orc, om, shape=(6, 7, 8))
    f = orc.rhs(om, U, (1e-4, 1.3e-4, 0.8e-4))
    sh = (2, 3, 5)
    fs = orc.rhs(om, np.roll(U, sh, axis=(1, 2, 3)), (1e-4, 1.3e-4, 0.8e-4))
    np.testing.assert_array_equal(fs, np.roll(f, sh, axis=(1, 2, 3)))
    # swap x and y: transpose the grid, exchange the momentum components
    Ut = np.swapaxes(U, 2, 3).copy()
    Ut[[1, 2]] = Ut[[2, 1]]
    ft = orc.rhs(om, Ut, (1.3e-4, 1e-4, 0.8e-4))
    ft[[1, 2]] = ft[[2, 1]]
    back = np.swapaxes(ft, 2, 3)
    for q in range(U.shape[0]):
        assert np.abs(back[q] - f[q]).max() <= 1e-12 * np.abs(f[q]).max(), q


# ---------------------------------------------------------------- spectral
def _sd(f, axis, dx):
    n = f.shape[axis]
    k = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    shape = [1] * f.ndim
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def _grad(f, dx):
    # axes of a [z][y][x] field: x = 2, y = 1, z = 0
    return [_sd(f, 2, dx), _sd(f, 1, dx), _sd(f, 0, dx)]


def _div(F, dx):
    return _sd(F[0], 2, dx) + _sd(F[1], 1, dx) + _sd(F[2], 0, dx)


def _smooth_fields(n, om, varying_T):
    L = n * 1e-4
    dx = 1e-4
    z, y, x = np.meshgrid(*(np.arange(n) * dx,) * 3, indexing="ij")
    kx = 2 * np.pi / L
    u = np.stack([3 * np.sin(kx * y) + 2 * np.cos(kx * (x + z)),
                  -2 * np.cos(kx * z) + np.sin(2 * kx * x),
                  np.sin(kx * (x - y)) + 1.5 * np.cos(kx * y)])
    if varying_T:
        T = 900 + 300 * np.sin(kx * x) * np.cos(kx * y) + 100 * np.cos(kx * z)
        Ya = np.random.default_rng(7).dirichlet(np.ones(om.ns))
        Yb = np.random.default_rng(8).dirichlet(np.ones(om.ns))
        w = 0.5 * (1 + np.sin(kx * (y + z)))
        Y = w * Ya[:, None, None, None] + (1 - w) * Yb[:, None, None, None]
        u = 0.0 * u
    else:
        T = np.full(x.shape, 1000.0)
        Y = np.broadcast_to(np.random.default_rng(7).dirichlet(np.ones(om.ns))[:, None, None, None],
                            (om.ns,) + x.shape).copy()
    p = np.full(x.shape, 101325.0)
    return dict(p=p, T=T, Y=Y, u=u), dx


def _rates(errs):
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("wide", [False, True])
def test_viscous_terms_converge_to_continuous_stress_divergence(orc, mechs, wide):
    om = mechs["mech9le"]        # bulk viscosity 0.6 mu exercises the xi terms
    if wide:                     # the wide stencil D(mu D u) of Section 2.2
        om = orc.Mechanism(om.mech, wide=True)
    m = om.mech
    errs_m, errs_e = [], []
    for n in (16, 32):
        prim, dx = _smooth_fields(n, om, varying_T=False)
        U = orc.prim_to_cons(om, prim)
        f = orc.rhs(om, U, dx, parts=orc.DIFF)
        mu = m["mu_ref"] * (1000.0 / m["T_ref"]) ** m["mu_exp"]
        xi = m["bulk_ratio"] * mu
        u = prim["u"]
        G = [_grad(u[i], dx) for i in range(3)]          # G[i][j] = d_j u_i
        divu = G[0][0] + G[1][1] + G[2][2]
        tau = [[mu * (G[i][j] + G[j][i]) + (xi - 2 * mu / 3) * divu * (i == j) for j in range(3)]
               for i in range(3)]
        divtau = [_div(tau[i], dx) for i in range(3)]
        work = _div([sum(tau[i][j] * u[j] for j in range(3)) for i in range(3)], dx)
        errs_m.append(max(np.abs(f[1 + i] - divtau[i]).max() / np.abs(divtau[i]).max() for i in range(3)))
        errs_e.append(np.abs(f[4] - work).max() / np.abs(work).max())
    # (the wide stencil's error constant is larger than the narrow one's)
    lim = 10.0 if wide else 1.0
    assert errs_m[-1] < 1e-6 * lim and errs_e[-1] < 1e-5 * lim, (errs_m, errs_e)
    assert _rates(errs_m)[0] > 7.0 and _rates(errs_e)[0] > 7.0, (errs_m, errs_e)


@pytest.mark.parametrize("wide", [False, True])
def test_diffusive_fluxes_converge_to_continuous_divergence(orc, mechs, wide):
    om = mechs["mech9le"]        # non-unity Lewis numbers: V_c is active
    if wide:
        om = orc.Mechanism(om.mech, wide=True)
    m = om.mech
    W = m["W"]
    errs = []
    for n in (16, 32):
        prim, dx = _smooth_fields(n, om, varying_T=True)
        U = orc.prim_to_cons(om, prim)
        f = orc.rhs(om, U, dx, parts=orc.DIFF)
        T, Y, p = prim["T"], prim["Y"], prim["p"]
        flatT = T.reshape(-1)
        cpR = np.zeros((om.ns, flatT.size))
        hRT = np.zeros_like(cpR)
        for c, Tc in enumerate(flatT):
            cpR[:, c], hRT[:, c], _ = orc.species_thermo(om, Tc)
        cpR = cpR.reshape((om.ns,) + T.shape)
        hRT = hRT.reshape((om.ns,) + T.shape)
        Wbar = 1.0 / np.sum(Y / W[:, None, None, None], axis=0)
        X = Y * Wbar / W[:, None, None, None]
        h = RU / W[:, None, None, None] * T * hRT
        cp = np.sum(Y * RU / W[:, None, None, None] * cpR, axis=0)
        mu = m["mu_ref"] * (T / m["T_ref"]) ** m["mu_exp"]
        lam = mu * cp / m["Pr"]
        rhoD = lam / cp / m["Le"][:, None, None, None]
        gp = _grad(p, dx)
        Fbar = [[-rhoD[k] * (gX + (X[k] - Y[k]) * gpd / p) for gX, gpd in zip(_grad(X[k], dx), gp)]
                for k in range(om.ns)]
        Vc = [sum(Fbar[k][d] for k in range(om.ns)) for d in range(3)]
        F = [[Fbar[k][d] - Y[k] * Vc[d] for d in range(3)] for k in range(om.ns)]
        species = [-_div(F[k], dx) for k in range(om.ns)]
        gT = _grad(T, dx)
        energy = _div([lam * gT[d] - sum(F[k][d] * h[k] for k in range(om.ns)) for d in range(3)], dx)
        e = [np.abs(f[5 + k] - species[k]).max() / np.abs(species[k]).max() for k in range(om.ns)]
        e.append(np.abs(f[4] - energy).max() / np.abs(energy).max())
        errs.append(max(e))
    assert errs[-1] < (1e-5 if wide else 1e-6), errs
    assert _rates(errs)[0] > 7.0, errs


@pytest.mark.parametrize("kind,ref", [("mech9le", 8), ("mech9le", 0)])
def test_reference_species_fluxes_converge_to_continuous_divergence(orc, mechs, kind, ref):
    """Reference-species form (Section 2.1): F_k = Fbar_k for k != ref, F_ref =
    -sum of the others; the energy flux is sum_k F_k h_k.  Eighth-order
    convergence to the spectral divergence of those fluxes, and species
    diffusion terms that sum to zero."""
    om0 = mechs[kind]
    om = orc.Mechanism(om0.mech, ref_species=ref)
    m = om.mech
    W = m["W"]
    errs = []
    for n in (16, 32):
        prim, dx = _smooth_fields(n, om, varying_T=True)
        U = orc.prim_to_cons(om, prim)
        f = orc.rhs(om, U, dx, parts=orc.DIFF)
        T, Y, p = prim["T"], prim["Y"], prim["p"]
        flatT = T.reshape(-1)
        cpR = np.zeros((om.ns, flatT.size))
        hRT = np.zeros_like(cpR)
        for c, Tc in enumerate(flatT):
            cpR[:, c], hRT[:, c], _ = orc.species_thermo(om, Tc)
        cpR = cpR.reshape((om.ns,) + T.shape)
        hRT = hRT.reshape((om.ns,) + T.shape)
        Wbar = 1.0 / np.sum(Y / W[:, None, None, None], axis=0)
        X = Y * Wbar / W[:, None, None, None]
        h = RU / W[:, None, None, None] * T * hRT
        cp = np.sum(Y * RU / W[:, None, None, None] * cpR, axis=0)
        mu = m["mu_ref"] * (T / m["T_ref"]) ** m["mu_exp"]
        lam = mu * cp / m["Pr"]
        rhoD = lam / cp / m["Le"][:, None, None, None]
        gp = _grad(p, dx)
        Fbar = [[-rhoD[k] * (gX + (X[k] - Y[k]) * gpd / p) for gX, gpd in zip(_grad(X[k], dx), gp)]
                for k in range(om.ns)]
        F = [Fbar[k] if k != ref else [-sum(Fbar[j][d] for j in range(om.ns) if j != ref) for d in range(3)]
             for k in range(om.ns)]
        species = [-_div(F[k], dx) for k in range(om.ns)]
        gT = _grad(T, dx)
        energy = _div([lam * gT[d] - sum(F[k][d] * h[k] for k in range(om.ns)) for d in range(3)], dx)
        e = [np.abs(f[5 + k] - species[k]).max() / np.abs(species[k]).max() for k in range(om.ns)]
        e.append(np.abs(f[4] - energy).max() / np.abs(energy).max())
        errs.append(max(e))
        tot = np.sum(f[5:], axis=0)
        assert np.abs(tot).max() <= 1e-12 * np.abs(f[5:]).max()
    assert errs[-1] < 1e-6
    assert _rates(errs)[0] > 7.0, errs
    # the two forms differ (the correction velocity is not zero here)
    f0 = orc.rhs(om0, U, dx, parts=orc.DIFF)
    assert np.abs(f0[5 + ref] - f[5 + ref]).max() > 1e-3 * np.abs(f[5 + ref]).max()


def test_wide_stencil_does_not_see_the_nyquist_mode(orc, mechs):
    """The wide operator D(lambda D T) differentiates twice with the centred
    first derivative, which is zero on the grid's odd-even (Nyquist) mode, so
    a temperature field T0 + eps (-1)^i gives no conduction term at all; the
    narrow operator damps that mode strongly (the reason for it, Section 2.2)."""
    om = mechs["mech9"]
    omw = orc.Mechanism(om.mech, wide=True)
    n = 8
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    T = 1000.0 + 5.0 * (-1.0) ** x
    Y = np.broadcast_to(np.random.default_rng(7).dirichlet(np.ones(om.ns))[:, None, None, None],
                        (om.ns, n, n, n)).copy()
    prim = dict(p=np.full(T.shape, 101325.0), T=T, Y=Y, u=np.zeros((3,) + T.shape))
    U = orc.prim_to_cons(om, prim)
    fw = orc.rhs(omw, U, 1e-4, parts=orc.DIFF)
    fn = orc.rhs(om, U, 1e-4, parts=orc.DIFF)
    assert np.abs(fn[4]).max() > 1e6
    assert np.abs(fw[4]).max() <= 1e-9 * np.abs(fn[4]).max()


def test_subset_mechanism_keeps_its_parents_data():
    """The 12-species mechanism is the 21-species one restricted to a species
    subset: every kept reaction appears in the parent with the same species
    (mapped by name) and the same Arrhenius triple, every parent reaction
    among the kept species is kept, and each reaction balances elements."""
    full, sub = mechanism.load("mech21"), mechanism.load("mech12")
    pos = [full["species"].index(s) for s in sub["species"]]
    parent = {}
    for j in range(full["nr"]):
        parent[(tuple(full["nu_f"][j]), tuple(full["nu_r"][j]))] = (full["A"][j], full["b"][j], full["Ea"][j])
    inside = 0
    for j in range(full["nr"]):
        used = (full["nu_f"][j] > 0) | (full["nu_r"][j] > 0)
        inside += all(used[k] == 0 or k in pos for k in range(full["ns"]))
    assert sub["nr"] == inside > 0
    for j in range(sub["nr"]):
        nf, nr_ = np.zeros(full["ns"], np.int32), np.zeros(full["ns"], np.int32)
        nf[pos], nr_[pos] = sub["nu_f"][j], sub["nu_r"][j]
        assert parent[(tuple(nf), tuple(nr_))] == (sub["A"][j], sub["b"][j], sub["Ea"][j])
        assert not ((sub["nu_r"][j] - sub["nu_f"][j]) @ sub["composition"]).any()
    np.testing.assert_array_equal(sub["W"], np.asarray(full["W"])[pos])
    np.testing.assert_array_equal(sub["nasa"], np.asarray(full["nasa"])[pos])
