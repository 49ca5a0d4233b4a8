"""Pins of the oracle's time step against closed forms, invariants and
special cases that reduce to textbook routines."""
import math

import numpy as np
import pytest

import lbm_inputs as li
from oracle import eos, moments, ref
from tests.golden_io import paper_values

Q = 19
E = np.array(moments.VELOCITIES)
W_STD = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


# ---------------------------------------------------------------------------
# Equation of state and pseudopotential
# ---------------------------------------------------------------------------
def test_maxwell_cs_printed_values():
    """Square-root psi with the C-S EOS at T = 0.6 T_c: the paper prints the
    Maxwell coexistence densities 0.406 / 0.00308 (Sec. IV.D)."""
    pv = paper_values()["maxwell_cs_T0.6Tc"]
    for a in (0.25, 0.5):  # a scales pressure only; coexistence is independent of it
        p = ref.make_params(li.params(1, 1, 1, T_over_Tc=0.6, eos_a=a))
        rl, rv = eos.maxwell(ref.pressure_fn(p), 1e-6, 0.99)
        assert round(rl, 3) == pv["rho_L"]
        assert round(rv, 5) == pv["rho_V"]


def test_maxwell_exponential_printed_values():
    """psi = psi0 exp(-rho0/rho), psi0 = rho0 = 1, G = -10/3: 2.783 / 0.3675
    (Sec. IV.A)."""
    pv = paper_values()["maxwell_exponential_G_-10/3"]
    p = ref.make_params(li.params(1, 1, 1, psi_form="exp", G=-10.0 / 3.0, psi0=1.0, rho0=1.0))
    rl, rv = eos.maxwell(ref.pressure_fn(p), 0.05, 20.0)
    assert round(rl, 3) == pv["rho_L"]
    assert round(rv, 4) == pv["rho_V"]


@pytest.mark.parametrize("t", [0.5, 0.6, 0.7, 0.8, 0.9])
def test_sqrt_psi_real_over_liquid_range(t):
    """With G = -1 the radicand stays positive from 0 to 1.2 rho_L."""
    p = ref.make_params(li.params(1, 1, 1, T_over_Tc=t))
    rl, _ = li.coexistence(t)
    r = np.linspace(1e-6, 1.2 * rl, 2001)
    assert np.all(np.isfinite(ref.psi(p, r)))
    assert np.all(ref.psi(p, r) > 0)


def test_coexistence_table_consistent_with_oracle():
    p = ref.make_params(li.params(1, 1, 1, T_over_Tc=0.7))
    rl, rv = eos.maxwell(ref.pressure_fn(p), 1e-6, 0.99)
    trl, trv = li.coexistence(0.7)
    assert abs(rl - trl) < 1e-10 and abs(rv - trv) < 1e-12


# ---------------------------------------------------------------------------
# Equilibria
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_rest_equilibrium_is_textbook_weights(op):
    p = ref.make_params(li.params(2, 2, 2, op=op))
    rho = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8])
    f = ref.equilibrium(p, rho, np.zeros((3, 8)))
    np.testing.assert_allclose(f, W_STD[:, None] * rho[None, :], rtol=4e-15, atol=0)


@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_equilibrium_recovers_rho_and_momentum(op):
    p = ref.make_params(li.params(4, 4, 4, op=op))
    rho, u = li.random_fields(4, 4, 4, seed=11, umax=0.1)
    f = ref.equilibrium(p, rho, u)
    np.testing.assert_allclose(f.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(E.T.astype(float) @ f, rho * u, rtol=1e-13, atol=1e-17)


# ---------------------------------------------------------------------------
# Equal-rate (BGK) reduction, brute force on 4^3
# ---------------------------------------------------------------------------
def _roll_to(field, e):
    """field(x + e) for a (nz, ny, nx) periodic array."""
    return np.roll(field, shift=(-e[2], -e[1], -e[0]), axis=(0, 1, 2))


def _bgk_step_reference(p_or, cfg, f, s, nonorth):
    """Independent velocity-space step for the all-rates-equal case:
    fbar* = fbar - s (fbar - f^B) + (1 - s/2) (G^B + X v4), then stream.
    Non-orthogonal: f^B = M^-1 m_eq, G^B = M^-1 S in closed form (derived by
    hand from Eqs. (13), (14) and Appendix A).  Orthogonal: textbook D3Q19
    equilibrium and the Guo forcing.  X v4 is the Eq. (16) term carried to
    velocity space: v4 = column 4 of M^-1 = (-1, 1/6 x 6, 0 x 12)."""
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    f4 = f.reshape(Q, nz, ny, nx)
    rho = f4.sum(0)
    psi = ref.psi(p_or, rho.reshape(-1)).reshape(rho.shape)
    acc = np.zeros((3,) + rho.shape)
    for a in range(1, Q):
        w = 1 / 6 if a <= 6 else 1 / 12
        pn = _roll_to(psi, E[a])
        for d in range(3):
            acc[d] += w * pn * E[a][d]
    G = cfg["G"]
    Fm = -G * psi[None] * acc
    F = Fm.copy()
    j = np.einsum("ad,azyx->dzyx", E.astype(float), f4)
    u = (j + 0.5 * F) / rho[None]
    u2 = (u * u).sum(0)
    uF = (u * F).sum(0)
    fB = np.empty_like(f4)
    GB = np.empty_like(f4)
    for a in range(Q):
        e = E[a]
        eu = sum(e[d] * u[d] for d in range(3))
        eF = sum(e[d] * F[d] for d in range(3))
        nzs = [d for d in range(3) if e[d] != 0]
        if nonorth:
            if a == 0:
                fB[a] = rho * (2 - 5 * u2) / 6
                GB[a] = -2.0 / 3.0 * uF
            elif len(nzs) == 1:
                fB[a] = rho * (1 + 3 * eu + 6 * eu * eu) / 18
                GB[a] = eF / 6 + 2.0 / 3.0 * eu * eF - uF / 3
            else:
                i_, j_ = nzs
                k_ = [d for d in range(3) if e[d] == 0][0]
                fB[a] = rho * (2 + 6 * eu + 9 * eu * eu - 6 * (u[i_] ** 2 + u[j_] ** 2) - 3 * u[k_] ** 2) / 72
                GB[a] = eF / 12 + eu * eF / 4 - (u[i_] * F[i_] + u[j_] * F[j_]) / 12
        else:
            fB[a] = W_STD[a] * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * u2)
            GB[a] = W_STD[a] * (3 * (eF - uF) + 9 * eu * eF)
    Fm2 = (Fm * Fm).sum(0)
    X = 6 * cfg["sigma"] * Fm2 / (psi * psi) / (1 / s - 0.5)
    if nonorth or cfg.get("orth_sigma", 0):
        v4 = np.array([-1.0] + [1 / 6] * 6 + [0.0] * 12)
    else:
        # orthogonal model with the term on its e row only (19 X there):
        # velocity-space image 19 X (19 |e|^2 - 30) / 2394 per direction
        e2 = (E * E).sum(1)
        v4 = 19.0 * (19.0 * e2 - 30.0) / 2394.0
    post = f4 - s * (f4 - fB) + (1 - s / 2) * (GB + v4[:, None, None, None] * X[None])
    out = np.empty_like(post)
    for a in range(Q):
        out[a] = np.roll(post[a], shift=(E[a][2], E[a][1], E[a][0]), axis=(0, 1, 2))
    return out.reshape(Q, -1)


@pytest.mark.parametrize("op", ["nonorth", "orth", "orth_sigma_e_eps"])
@pytest.mark.parametrize("s", [1.3, 0.8])
def test_equal_rates_reduce_to_bgk(op, s):
    """With all rates equal, each operator is a BGK step with Guo forcing plus
    the Eq. (16) term carried to velocity space.  The orthogonal model with
    the term on its e and eps rows applies exactly the non-orthogonal
    correction; with the term on e only (the default reading) its image is
    19 X (19 |e|^2 - 30) / 2394."""
    cfg = li.params(4, 4, 4, op=op.split("_")[0], T_over_Tc=0.8, sigma=0.105, rates=[s] * Q,
                    orth_sigma=1 if op.endswith("e_eps") else 0)
    p = ref.make_params(cfg)
    f = li.random_populations(4, 4, 4, seed=7, lo=0.0005, hi=0.02)
    got = ref.step(p, f, 1)
    want = _bgk_step_reference(p, cfg, f, s, op == "nonorth")
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-16)
    if op != "nonorth":  # the two orthogonal readings differ by the eps-row term
        other = _bgk_step_reference(p, dict(cfg, orth_sigma=1 - cfg["orth_sigma"]), f, s, False)
        assert not np.allclose(got, other, rtol=1e-10, atol=0)


def test_bgk_reference_rejects_planted_error():
    """The brute-force comparison is sensitive: a single wrong equilibrium
    coefficient (planted in the reference) is detected."""
    cfg = li.params(4, 4, 4, T_over_Tc=0.8, sigma=0.105, rates=[1.3] * Q)
    p = ref.make_params(cfg)
    f = li.random_populations(4, 4, 4, seed=7, lo=0.0005, hi=0.02)
    got = ref.step(p, f, 1)
    bad = _bgk_step_reference(p, dict(cfg, sigma=0.1), f, 1.3, True)
    assert not np.allclose(got, bad, rtol=1e-10, atol=0)


# ---------------------------------------------------------------------------
# Conservation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_mass_and_momentum_conservation_periodic(op):
    """Mass is conserved exactly (columns of M^-1 sum to delta_k0) and, with no
    body force, the bare momentum sum_x sum_a e_a fbar_a is conserved because
    sum_x F_m = 0 on a periodic lattice (pairwise antisymmetry of Eq. (15))."""
    cfg, init = li.c3_two_droplets(n=24, op=op)
    p = ref.make_params(cfg)
    rho, u = li.init_fields(cfg, init)
    f0 = ref.equilibrium(p, rho, u)
    f1 = ref.step(p, f0, 60)
    m0, m1 = f0.sum(), f1.sum()
    assert abs(m1 - m0) / m0 < 1e-13
    P0 = E.T.astype(float) @ f0.sum(1)
    P1 = E.T.astype(float) @ f1.sum(1)
    assert np.all(np.abs(P1 - P0) < 1e-13 * m0)
    fl = ref.fields(p, f1)
    assert np.abs(fl["F"].sum(1)).max() < 1e-13 * np.abs(fl["F"]).sum()


def test_mass_conservation_walls_gravity():
    cfg, init = li.c4_sessile(theta_deg=60.0, nx=24, ny=20, nz=16, r0=6.0)
    p = ref.make_params(cfg)
    rho, u = li.init_fields(cfg, init)
    f0 = ref.equilibrium(p, rho, u)
    f1 = ref.step(p, f0, 40)
    assert abs(f1.sum() - f0.sum()) / f0.sum() < 1e-13
    assert np.all(np.isfinite(f1))


def test_uniform_rest_state_is_fixed_point_with_walls():
    """A uniform fluid at rest between wetting walls: the Eq. (57) ghost layer
    equals the bulk (zero in-plane gradient) so F_m vanishes and the rest
    equilibrium is reproduced exactly by collision, streaming and bounce-back."""
    cfg = li.params(6, 5, 7, T_over_Tc=0.7, wall_z=1, theta_wall_deg=60.0)
    p = ref.make_params(cfg)
    rho = np.full(6 * 5 * 7, 0.2)
    f0 = ref.equilibrium(p, rho, np.zeros((3, rho.size)))
    f1 = ref.step(p, f0, 5)
    np.testing.assert_allclose(f1, f0, rtol=1e-14)


# ---------------------------------------------------------------------------
# Cube symmetry: the step commutes with the 48 lattice symmetries
# ---------------------------------------------------------------------------
def _transform(f, n, perm, signs):
    """Apply x' = S P x to a (19, n^3) state on an n^3 periodic lattice."""
    T = np.zeros((3, 3), dtype=int)
    for i in range(3):
        T[i, perm[i]] = signs[i]
    Et = E @ T.T
    vmap = [next(b for b in range(Q) if tuple(E[b]) == tuple(Et[a])) for a in range(Q)]
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()])
    newpos = (T @ pos) % n
    newidx = (newpos[2] * n + newpos[1]) * n + newpos[0]
    g = np.empty_like(f)
    for a in range(Q):
        g[vmap[a], newidx] = f[a]
    return g


@pytest.mark.parametrize("op", ["nonorth", "orth"])
@pytest.mark.parametrize("perm,signs", [((1, 0, 2), (1, 1, 1)), ((1, 2, 0), (1, 1, 1)),
                                        ((0, 1, 2), (-1, 1, 1))])
def test_step_equivariant_under_cube_symmetries(op, perm, signs):
    n = 6
    cfg = li.params(n, n, n, op=op, T_over_Tc=0.8, sigma=0.105)
    p = ref.make_params(cfg)
    rho, u = li.random_fields(n, n, n, seed=3, rho_lo=0.03, rho_hi=0.3, umax=0.05)
    f = ref.equilibrium(p, rho, u) * (1 + 0.1 * li.random_populations(n, n, n, seed=4, lo=-1, hi=1))
    a = _transform(ref.step(p, f, 2), n, perm, signs)
    b = ref.step(p, _transform(f, n, perm, signs), 2)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-17)


# ---------------------------------------------------------------------------
# Transport coefficients, Eq. (54)
# ---------------------------------------------------------------------------
def _single_phase(nx, ny, nz, op, s_e, s_nu, **kw):
    return li.params(nx, ny, nz, op=op, psi_form="exp", G=0.0, sigma=0.0, s_e=s_e,
                     tau_nu=1.0 / s_nu, **kw)


@pytest.mark.parametrize("op", ["nonorth", "orth", "orth_meq1"])
def test_shear_wave_decay_matches_eq54(op):
    """u_x = U sin(k y) decays at nu k^2 with nu = c_s^2 (1/s_nu - 1/2); for
    the orthogonal operator also with the other equilibrium reading (the
    stress rows, which set the shear viscosity, are the same)."""
    L, s_nu = 64, 1.2
    cfg = _single_phase(1, L, 1, op.split("_")[0], s_e=0.9, s_nu=s_nu)
    cfg["orth_meq"] = 1 if op.endswith("meq1") else 0
    p = ref.make_params(cfg)
    k = 2 * math.pi / L
    y = np.arange(L)
    u = np.zeros((3, L))
    u[0] = 1e-4 * np.sin(k * y)
    f = ref.equilibrium(p, np.ones(L), u)
    f = ref.step(p, f, 50)
    a1 = (ref.fields(p, f)["u"][0] * np.sin(k * y)).sum()
    f = ref.step(p, f, 300)
    a2 = (ref.fields(p, f)["u"][0] * np.sin(k * y)).sum()
    nu_meas = -math.log(a2 / a1) / (k * k * 300)
    nu = (1 / s_nu - 0.5) / 3
    assert abs(nu_meas / nu - 1) < 0.01


@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_sound_wave_damping_matches_eq54(op):
    """A standing sound wave decays at k^2 (4 nu / 3 + nu_b) / 2 with
    mu_b = (2/3) rho c_s^2 (1/s_e - 1/2) (Eq. (54), Eq. (56))."""
    L, s_e, s_nu = 64, 0.8, 1.25
    cfg = _single_phase(L, 1, 1, op, s_e=s_e, s_nu=s_nu)
    p = ref.make_params(cfg)
    k = 2 * math.pi / L
    x = np.arange(L)
    f = ref.equilibrium(p, 1 + 1e-5 * np.cos(k * x), np.zeros((3, L)))

    def energy(f):
        fl = ref.fields(p, f)
        rc = (fl["rho"] * np.cos(k * x)).sum() * 2 / L
        js = (fl["rho"] * fl["u"][0] * np.sin(k * x)).sum() * 2 / L
        return rc * rc + 3.0 * js * js  # rho'^2 + (j / c_s)^2

    f = ref.step(p, f, 40)
    e1 = energy(f)
    f = ref.step(p, f, 400)
    e2 = energy(f)
    gamma = -math.log(e2 / e1) / (2 * 400)
    nu = (1 / s_nu - 0.5) / 3
    nub = (2.0 / 3.0) * (1 / s_e - 0.5) / 3
    want = k * k * (4 * nu / 3 + nub) / 2
    assert abs(gamma / want - 1) < 0.03


def test_poiseuille_between_bounce_back_walls():
    """Body force rho g_x between half-way walls at z = -1/2 and nz - 1/2:
    the steady profile is g (z + 1/2)(nz - 1/2 - z) / (2 nu)."""
    nz, gx, s_nu = 24, 1e-6, 1.0
    cfg = _single_phase(1, 1, nz, "nonorth", s_e=1.1, s_nu=s_nu, wall_z=1, gravity=(gx, 0.0, 0.0))
    p = ref.make_params(cfg)
    f = ref.equilibrium(p, np.ones(nz), np.zeros((3, nz)))
    f = ref.step(p, f, 12000)
    ux = ref.fields(p, f)["u"][0]
    z = np.arange(nz)
    nu = (1 / s_nu - 0.5) / 3
    want = gx * (z + 0.5) * (nz - 0.5 - z) / (2 * nu)
    assert np.abs(ux - want).max() < 0.01 * want.max()


# ---------------------------------------------------------------------------
# Sampled step (used for parity on full-size lattices) equals the full step
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("walls", [False, True])
def test_step_sampled_equals_full_step(walls):
    if walls:
        cfg, init = li.c4_sessile(theta_deg=120.0, nx=10, ny=9, nz=8, r0=3.0)
    else:
        cfg, init = li.c3_two_droplets(n=12)
    p = ref.make_params(cfg)
    rho, u = li.init_fields(cfg, init)
    f0 = ref.equilibrium(p, rho, u)
    full = ref.step(p, f0, 1)
    idx = np.arange(f0.shape[1])
    samp = ref.step_sampled(p, f0, idx)
    np.testing.assert_array_equal(samp.T, full)


# ---------------------------------------------------------------------------
# Density-dependent viscosity (the reading of the nu_V / nu_L runs of Sec. IV.D:
# nu linear in rho between visc_rho_V and visc_rho_L, constant outside).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_variable_viscosity_shear_wave_at_mid_density(op):
    """At a uniform density halfway between visc_rho_V and visc_rho_L the
    shear wave decays at the mean of nu_L and nu_V (Eq. (54))."""
    L, s_nu, ratio = 64, 1.6, 4.0
    nu_L = (1 / s_nu - 0.5) / 3
    cfg = _single_phase(1, L, 1, op, s_e=0.9, s_nu=s_nu)
    cfg.update(nu_ratio=ratio, visc_rho_L=1.5, visc_rho_V=0.5)
    p = ref.make_params(cfg)
    k = 2 * math.pi / L
    y = np.arange(L)
    u = np.zeros((3, L))
    u[0] = 1e-4 * np.sin(k * y)
    f = ref.equilibrium(p, np.ones(L), u)
    f = ref.step(p, f, 50)
    a1 = (ref.fields(p, f)["u"][0] * np.sin(k * y)).sum()
    f = ref.step(p, f, 200)
    a2 = (ref.fields(p, f)["u"][0] * np.sin(k * y)).sum()
    nu_meas = -math.log(a2 / a1) / (k * k * 200)
    assert abs(nu_meas / (0.5 * (nu_L + ratio * nu_L)) - 1) < 0.01


@pytest.mark.parametrize("op", ["nonorth", "orth"])
@pytest.mark.parametrize("side", ["vapour", "liquid"])
def test_variable_viscosity_reduces_to_constant_rates_outside_range(op, side):
    """Below visc_rho_V every node relaxes the stress rows at the rate of
    nu_V = ratio nu_L, above visc_rho_L at s_nu: one step equals a
    constant-rate step with that rate."""
    s_nu, ratio = 1.5, 3.0
    nu_V = ratio * (1 / s_nu - 0.5) / 3
    rho, u = li.random_fields(4, 5, 3, seed=3, rho_lo=0.1, rho_hi=0.3)
    if side == "liquid":
        rho = rho + 1.0
    cfg = dict(li.params(4, 5, 3, op=op, s_nu=s_nu), G=-1.0)
    cfg.pop("tau_nu", None)
    var = dict(cfg, nu_ratio=ratio, visc_rho_L=1.0, visc_rho_V=0.35)
    const = dict(cfg, s_nu=1 / (3 * nu_V + 0.5) if side == "vapour" else s_nu)
    pv, pc = ref.make_params(var), ref.make_params(const)
    f0 = ref.equilibrium(pc, rho, u) * (1 + 0.02 * li.random_populations(4, 5, 3, 4, -1, 1))
    a = ref.step(pv, f0, 1)
    b = ref.step(pc, f0, 1)
    assert np.allclose(a, b, rtol=1e-14, atol=0)


# ---------------------------------------------------------------------------
# Single-phase walls on x and y and the moving lid (lid-driven cavity of
# Appendix B)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_plane_couette_flow_is_linear(op):
    """Walls at y = -1/2 (fixed) and ny - 1/2 (moving at U along x): the
    steady profile is u_x = U (y + 1/2) / ny, which half-way bounce-back
    reproduces to rounding for the non-orthogonal model; the orthogonal
    model's u^2 terms perturb the density at O(U^2) and the profile by
    about 1e-7 U.  A wall misplaced by half a node would be off by ~3 %."""
    ny, U = 16, 0.01
    cfg = _single_phase(1, ny, 1, op, s_e=1.1, s_nu=1.0, wall_y=1, lid_u=(U, 0.0, 0.0))
    p = ref.make_params(cfg)
    f = ref.equilibrium(p, np.ones(ny), np.zeros((3, ny)))
    f = ref.step(p, f, 20000)
    fl = ref.fields(p, f)
    y = np.arange(ny)
    np.testing.assert_allclose(fl["u"][0], U * (y + 0.5) / ny, rtol=0, atol=(1e-9 if op == "nonorth" else 1e-6) * U)
    np.testing.assert_allclose(fl["u"][1:], 0.0, atol=1e-12)


def test_plane_couette_flow_reverses_with_the_lid():
    """The sign of the lid term: a lid moving along -x drives -u_x."""
    ny, U = 8, 0.01
    cfg = _single_phase(1, ny, 1, "nonorth", s_e=1.1, s_nu=1.2, wall_y=1, lid_u=(-U, 0.0, 0.0))
    p = ref.make_params(cfg)
    f = ref.step(p, ref.equilibrium(p, np.ones(ny), np.zeros((3, ny))), 6000)
    assert np.all(ref.fields(p, f)["u"][0] < 0)


@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_poiseuille_between_x_walls(op):
    """Body force rho g_z between half-way walls at x = -1/2 and nx - 1/2:
    g (x + 1/2)(nx - 1/2 - x) / (2 nu)."""
    nx, gz, s_nu = 24, 1e-6, 1.0
    cfg = _single_phase(nx, 1, 1, op, s_e=1.1, s_nu=s_nu, wall_x=1, gravity=(0.0, 0.0, gz))
    p = ref.make_params(cfg)
    f = ref.step(p, ref.equilibrium(p, np.ones(nx), np.zeros((3, nx))), 12000)
    uz = ref.fields(p, f)["u"][2]
    x = np.arange(nx)
    nu = (1 / s_nu - 0.5) / 3
    want = gz * (x + 0.5) * (nx - 0.5 - x) / (2 * nu)
    assert np.abs(uz - want).max() < 0.01 * want.max()


@pytest.mark.parametrize("op", ["nonorth", "orth"])
def test_closed_cavity_conserves_mass_and_z_mirror_symmetry(op):
    """Walls on all six faces, lid moving along x: mass is conserved (the lid
    terms of opposite x-directions cancel) and the flow stays symmetric
    under z -> nz - 1 - z."""
    nx, ny, nz = 7, 6, 5
    cfg = _single_phase(nx, ny, nz, op, s_e=1.1, s_nu=1.3, wall_x=1, wall_y=1, wall_z=1,
                        lid_u=(0.05, 0.0, 0.0))
    p = ref.make_params(cfg)
    N = nx * ny * nz
    f0 = ref.equilibrium(p, np.ones(N), np.zeros((3, N)))
    f = ref.step(p, f0, 200)
    assert abs(f.sum() - f0.sum()) < 1e-13 * f0.sum()
    u = ref.fields(p, f)["u"].reshape(3, nz, ny, nx)
    np.testing.assert_allclose(u[0], u[0][::-1], atol=1e-14)
    np.testing.assert_allclose(u[2], -u[2][::-1], atol=1e-14)
    assert u[0][:, -1, :].mean() > 0 > u[0][:, 0, :].mean()  # driven near the lid, return flow below


def test_low_viscosity_diverges_within_bounded_steps():
    """Failure detection on the CPU, at T = 0.5 T_c (density ratio about
    724, where Sec. IV.A reports instability at small viscosity): s_nu = 1.9
    (nu = 0.0088) blows up to non-finite populations within 100 steps, while
    s_nu = 1 (nu = 1/6) stays finite over 1000 steps with its spurious
    currents decaying below 0.01."""
    for s_nu, steps in ((1.9, 100), (1.0, 1000)):
        cfg, init = li.cold_droplet(s_nu)
        p = ref.make_params(cfg)
        f = ref.equilibrium(p, *li.init_fields(cfg, init))
        first_bad = None
        for k in range(0, steps, 10):
            f = ref.step(p, f, 10)
            if not np.isfinite(f).all():
                first_bad = k + 10
                break
        if s_nu > 1.5:
            assert first_bad is not None and first_bad <= 100
        else:
            assert first_bad is None
            u = ref.fields(p, f)["u"]
            assert float(np.sqrt((u ** 2).sum(0)).max()) < 0.01
