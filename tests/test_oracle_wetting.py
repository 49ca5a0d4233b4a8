"""Pins of the oracle's wetting ghost layer (Sec. IV.C, Eq. (57)).

Eq. (57) is the geometric contact-angle condition written as centred
differences about the first fluid layer: the normal difference
(rho_layer2 - rho_ghost) / 2 equals -cot(theta_a) times the in-plane gradient
magnitude phi / 2 of the first layer (phi: unhalved central differences), so
the isolines of density meet the wall at theta_a measured through the liquid.
Its defining property: a density field that already satisfies that condition
about the first layer is continued exactly.  The fields used here are

    rho = rho_0 - k sin(theta) (1 + kappa d^2) (n_t . r) - k cos(theta) d,

with n_t a unit vector in the wall plane and d the distance from the first
fluid layer into the fluid.  At d = 0 the gradient points into the liquid at
the angle theta to the wall; the kappa term is even in d, so it leaves the
centred normal difference alone but makes the in-plane gradient of the second
layer differ from the first.  The ghost value the rule must give is the same
formula at d = -1.  The pins compare the oracle's interaction force on the
first layer at both walls with the force that the oracle's periodic
(wall-free) code computes when the ghost layers are real fluid layers holding
that continuation, so the Eq. (57) code is checked against geometry rather
than against a retyping of itself.  Variant oracle libraries with a planted
mistake in each term of Eq. (57) are built on the CPU and shown to fail the
same comparison.
"""
import math
import os

import numpy as np
import pytest

import lbm_inputs as li
from oracle import build as obuild
from oracle import ref

NX, NY, NZ = 16, 14, 6
LO = 2  # nodes with x, y in [LO, n - 1 - LO] see no periodic seam of the field


def _contact_field(theta_deg, nz_layers, k=0.006, rho0=0.2, gamma_deg=30.0, kappa=0.5):
    """rho on layers z = -1 ... nz (nz_layers = nz + 2 values along z, layer
    index z + 1), meeting the walls z = -1/2 and z = nz - 1/2 at theta through
    the liquid.  d(z) = min(z, nz - 1 - z)."""
    nz = nz_layers - 2
    th = math.radians(theta_deg)
    g = math.radians(gamma_deg)
    x = np.arange(NX, dtype=np.float64)[None, None, :] - NX / 2
    y = np.arange(NY, dtype=np.float64)[None, :, None] - NY / 2
    z = np.arange(-1, nz + 1, dtype=np.float64)[:, None, None]
    d = np.minimum(z, nz - 1 - z)
    along = math.cos(g) * x + math.sin(g) * y
    return rho0 - k * math.sin(th) * (1.0 + kappa * d * d) * along - k * math.cos(th) * d


def _forces(theta_deg, ghost_rho_min=0.0, L=None, tan_wall=None):
    """(F of the walled lattice at z = 0 and nz - 1, F of the extended
    periodic lattice at the same nodes), each shape (2, 3, NY, NX)."""
    rho_ext = _contact_field(theta_deg, NZ + 2)
    # The two ghost layers, with the clamp of the rule applied.
    rho_ext[0] = np.maximum(rho_ext[0], ghost_rho_min)
    rho_ext[-1] = np.maximum(rho_ext[-1], ghost_rho_min)
    zeros = lambda n: np.zeros((3, n))  # noqa: E731

    cfg_w = li.params(NX, NY, NZ, T_over_Tc=0.7, wall_z=1, theta_wall_deg=float(theta_deg),
                      ghost_rho_min=float(ghost_rho_min))
    pw = ref.make_params(cfg_w)
    if tan_wall is not None:
        pw.tan_wall = tan_wall
    rho_w = np.ascontiguousarray(rho_ext[1:-1]).reshape(-1)
    fw = ref.equilibrium(pw, rho_w, zeros(rho_w.size))
    Fw = ref.fields(pw, fw, L=L)["F"].reshape(3, NZ, NY, NX)

    cfg_e = li.params(NX, NY, NZ + 2, T_over_Tc=0.7)
    pe = ref.make_params(cfg_e)
    rho_e = np.ascontiguousarray(rho_ext).reshape(-1)
    fe = ref.equilibrium(pe, rho_e, zeros(rho_e.size))
    Fe = ref.fields(pe, fe)["F"].reshape(3, NZ + 2, NY, NX)

    assert np.isfinite(Fw).all() and np.isfinite(Fe).all()
    got = np.stack([Fw[:, 0], Fw[:, NZ - 1]])
    want = np.stack([Fe[:, 1], Fe[:, NZ]])
    return got, want


def _window(a):
    return a[..., LO:NY - LO, LO:NX - LO]


def _rel_err(got, want):
    g, w = _window(got), _window(want)
    return np.abs(g - w).max() / np.abs(w).max()


@pytest.mark.parametrize("theta", [30.0, 60.0, 90.0, 120.0, 135.0])
def test_ghost_layer_continues_a_planar_contact_line(theta):
    """Both walls: the force on the first fluid layer equals the force with
    the exact linear continuation beyond the wall (Eq. (57))."""
    got, want = _forces(theta)
    assert _rel_err(got, want) < 1e-12
    if theta != 90.0:
        # The wetting layer matters here: the normal force on the first layer
        # comes from the ghost density differing from the layer above.
        assert np.abs(_window(want)[:, 2]).max() > 1e-4


def test_ghost_layer_clamp():
    """theta = 120 deg drives the continuation below layer 1; with the lower
    clamp set inside the range of ghost values, the clamped nodes see exactly
    the clamp density and the others the continuation."""
    rho_ext = _contact_field(120.0, NZ + 2)
    rmin = 0.2
    ghosts = np.stack([rho_ext[0], rho_ext[-1]])[..., LO:NY - LO, LO:NX - LO]
    assert (ghosts < rmin).any() and (ghosts > rmin).any()
    got, want = _forces(120.0, ghost_rho_min=rmin)
    assert _rel_err(got, want) < 1e-12
    unclamped, _ = _forces(120.0)
    assert _rel_err(got, unclamped) > 1e-6


_PLANTS = {1: "phi halved", 2: "layer 1 in place of layer 2", 3: "phi taken on layer 2",
           4: "sign of the phi term flipped"}


@pytest.fixture(scope="module")
def planted_libs(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_plants")
    return {k: ref.load(obuild.build(defines={"ORACLE_PLANT": k}, out=os.path.join(d, f"plant{k}.so")))
            for k in _PLANTS}


@pytest.mark.parametrize("plant", sorted(_PLANTS))
@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_ghost_layer_pin_rejects_planted_mistakes(planted_libs, plant, theta):
    got, want = _forces(theta, L=planted_libs[plant])
    assert _rel_err(got, want) > 1e-6, _PLANTS[plant]


@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_ghost_layer_pin_rejects_tan_theta(theta):
    """tan(theta) in place of tan(90 deg - theta) in the parameter mapping."""
    got, want = _forces(theta, tan_wall=math.tan(math.radians(theta)))
    assert _rel_err(got, want) > 1e-6
