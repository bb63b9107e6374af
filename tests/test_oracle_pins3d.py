"""Pins of the three-dimensional oracle (D3Q19 and D3Q27 lattices) against
what the paper and the mathematics fix.  Eq. (24) and Eq. (26) are written
for general dimension D; here D = 3, on either lattice.  As for two
dimensions, no test retypes the oracle's formulas: they check the lattice
weights' isotropy, moment identities, stencil exactness and reductions,
conservation, symmetries, a closed-form viscosity and the well-balanced fixed
point of the flat interface, solved independently."""
import numpy as np
import pytest

from paper_2012_11075_amd import inputs as I
from equilibrium import flat_equilibrium

# D3Q19 (the test's own copy): rest, 6 axis directions, 12 edge directions;
# D3Q27 adds the 8 corner directions
C19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
                [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)
C27 = np.concatenate([C19, [[1, 1, 1], [-1, -1, -1], [1, 1, -1], [-1, -1, 1],
                            [1, -1, 1], [-1, 1, -1], [-1, 1, 1], [1, -1, -1]]])
LATTICES = {19: C19, 27: C27}
CS2 = 1.0 / 3.0
SCHEMES = ["standard", "well_balanced"]
STEP_SCHEMES = SCHEMES + ["standard_eq_forcing"]


@pytest.fixture(params=[19, 27], ids=["d3q19", "d3q27"])
def q(request):
    return request.param


def test_velocity_sets_are_the_oracles(orc):
    assert np.array_equal(orc.C3, C19.astype(int))
    assert np.array_equal(orc.C27, C27.astype(int))
    # every velocity appears once, with its opposite
    for C in (C19, C27):
        assert len({tuple(c) for c in C}) == len(C)
        assert all(any((d == -c).all() for d in C) for c in C)


def test_lattice_weights_from_the_moments(orc, q):
    """The weights follow from the equilibrium at rest (feq_i(rho, 0) =
    w_i rho for the standard LBE), and they are the ones that make the
    lattice isotropic to fourth order: sum w = 1, sum w c c = cs2 I,
    sum w c_a c_b c_g c_d = cs2^2 (d_ab d_gd + d_ag d_bd + d_ad d_bg)."""
    C = LATTICES[q]
    p = orc.Params(0.8, 0.1, 0.02, 1.0, 0.1)
    w = orc.feq3("standard", p, 1.0, 0.0, 0.0, 0.0, q=q)
    d = np.eye(3)
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, C, C), CS2 * d, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, C, C, C, C)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(m4, iso, atol=1e-15)
    # the shells: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216
    shell = (C * C).sum(axis=1)
    want = {19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}, 27: {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}}[q]
    np.testing.assert_allclose(w, [want[s] for s in shell], rtol=1e-15)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("rho0", [0.0, 0.3])
def test_equilibrium_moments3(orc, scheme, rho0, q):
    """feq moments in 3-D: mass, momentum, cs2 rho I + rho uu (standard; WB:
    cs2 rho0 I + rho uu, Eq. 27 for D = 3) and the third moment
    cs2 rho (u d + d u + ..), which needs the lattice's fourth-order isotropy."""
    C = LATTICES[q]
    p = orc.Params(0.8, 0.1, 0.02, 1.0, 0.1, rho0)
    rng = np.random.default_rng(5)
    d = np.eye(3)
    for _ in range(40):
        rho = rng.uniform(0.05, 2.0)
        u = rng.uniform(-0.2, 0.2, 3)
        f = orc.feq3(scheme, p, rho, *u, q=q)
        iso = CS2 * (rho if scheme == "standard" else rho0)
        assert abs(f.sum() - rho) < 1e-14
        np.testing.assert_allclose(C.T @ f, rho * u, atol=1e-14)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", f, C, C),
                                   iso * d + rho * np.outer(u, u), atol=1e-14)
        m3 = np.einsum("i,ia,ib,ic->abc", f, C, C, C)
        uI = (np.einsum("a,bc->abc", u, d) + np.einsum("b,ac->abc", u, d)
              + np.einsum("c,ab->abc", u, d))
        np.testing.assert_allclose(m3, CS2 * rho * uI, atol=1e-14)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_forcing_moments3(orc, scheme, q):
    """F_i moments in 3-D: sum 0, first moment F, second moment uF + Fu, plus
    cs2 (u g + g u + (u.g) I) for Eq. (26) (G = F + cs2 grad rho and the
    (|c|^2/cs2 - D) term with D = 3)."""
    C = LATTICES[q]
    rng = np.random.default_rng(6)
    for _ in range(40):
        u = rng.uniform(-0.2, 0.2, 3)
        F = rng.uniform(-0.1, 0.1, 3)
        g = rng.uniform(-0.5, 0.5, 3)
        Fi = orc.forcing3(scheme, u, F, g, q=q)
        want = np.outer(u, F) + np.outer(F, u)
        if scheme == "well_balanced":
            want = want + CS2 * (np.outer(u, g) + np.outer(g, u) + np.dot(u, g) * np.eye(3))
        assert abs(Fi.sum()) < 1e-15
        np.testing.assert_allclose(C.T @ Fi, F, atol=1e-15)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", Fi, C, C), want, atol=1e-15)


def test_eq_forcing_moments3(orc, q):
    """The 3-D form of the forcing term named after Eq. (5),
    F_i = (c_i - u).F feq_i/(cs2 rho): from the moments of the equilibrium
    (second cs2 rho I + rho uu, third cs2 rho (u d)_sym, which the lattice's
    fourth-order isotropy gives), sum F_i = 0, sum c F_i = F and
    sum cc F_i = uF + Fu - uu (u.F)/cs2; F_i does not depend on rho."""
    C = LATTICES[q]
    rng = np.random.default_rng(16)
    p = orc.Params(0.8, 0.1, 0.02, 1.0, 0.1)
    for _ in range(40):
        rho = rng.uniform(0.05, 2.0)
        u = rng.uniform(-0.2, 0.2, 3)
        F = rng.uniform(-0.1, 0.1, 3)
        Fi = orc.forcing_eq3(p, rho, u, F, q=q)
        want = np.outer(u, F) + np.outer(F, u) - np.outer(u, u) * np.dot(u, F) / CS2
        assert abs(Fi.sum()) < 1e-15
        np.testing.assert_allclose(C.T @ Fi, F, atol=1e-15)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", Fi, C, C), want, atol=1e-15)
        np.testing.assert_allclose(orc.forcing_eq3(p, 2.5 * rho, u, F, q=q), Fi, atol=1e-16)


def test_stencils3_exact_on_quadratics_and_reduce_to_1d(orc, q):
    """The 3-D isotropic gradient and Laplacian are exact for quadratics
    (away from the seam), and on a field that varies along one axis they are
    the central difference and the 3-point Laplacian."""
    n = 14
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    phi = (0.2 + 0.01 * x - 0.02 * y + 0.03 * z + 0.001 * x * x - 0.002 * y * z
           + 0.0015 * z * z + 0.0005 * x * y)
    gx, gy, gz = orc.gradient3(phi, q=q)
    lap = orc.laplacian3(phi, q=q)
    s = (slice(2, n - 2),) * 3
    np.testing.assert_allclose(gx[s], (0.01 + 0.002 * x + 0.0005 * y)[s], atol=1e-13)
    np.testing.assert_allclose(gy[s], (-0.02 - 0.002 * z + 0.0005 * x)[s], atol=1e-13)
    np.testing.assert_allclose(gz[s], (0.03 - 0.002 * y + 0.003 * z)[s], atol=1e-13)
    np.testing.assert_allclose(lap[s], 0.002 + 0.003, atol=1e-13)
    prof = np.random.default_rng(2).normal(size=11)
    for axis in range(3):
        shape = [3, 3, 3]
        shape[axis] = 11
        field = np.broadcast_to(prof.reshape([-1 if a == axis else 1 for a in range(3)]), shape).copy()
        g = orc.gradient3(field, q=q)[2 - axis]   # (gx, gy, gz) vs array axes (z, y, x)
        lp = orc.laplacian3(field, q=q)
        cen = (np.roll(field, -1, axis) - np.roll(field, 1, axis)) / 2
        three = np.roll(field, -1, axis) - 2 * field + np.roll(field, 1, axis)
        np.testing.assert_allclose(g, cen, atol=1e-14)
        np.testing.assert_allclose(lp, three, atol=1e-14)


def droplet3(n, R, ph, width=4.0, noise=0.0, seed=1):
    c = n // 2
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    rho = 0.5 * (ph.rho_l + ph.rho_v) - 0.5 * (ph.rho_l - ph.rho_v) * np.tanh(2 * (r - R) / width)
    if noise:
        rho = rho * (1 + noise * np.random.default_rng(seed).uniform(-1, 1, rho.shape))
    return rho


@pytest.mark.parametrize("scheme", STEP_SCHEMES)
def test_mass_conservation_and_uniform_fixed_point3(orc, scheme, q):
    ph = I.PAPER_PHYS
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v)
    f = orc.init3(scheme, p, droplet3(12, 3.5, ph, noise=1e-2), q=q)
    m0 = orc.observe3(scheme, p, f)["mass"]
    f = orc.step3(scheme, p, f, 60)
    ob = orc.observe3(scheme, p, f)
    assert not ob["nonfinite"] and abs(ob["mass"] - m0) < 1e-12 * m0
    u = orc.init3(scheme, p, np.full((4, 5, 6), 0.7), q=q)
    v = orc.step3(scheme, p, u, 3)
    assert np.abs(u - v).max() <= 1e-15


# index of the population whose velocity is transform(c_i)
def _index_map(C, transform):
    out = []
    for c in C:
        t = transform(c)
        out.append(int(np.where((C == t).all(axis=1))[0][0]))
    return out


@pytest.mark.parametrize("scheme", STEP_SCHEMES)
def test_translation_permutation_and_mirror3(orc, scheme, q):
    """The step commutes with translations (bit for bit), with a cyclic
    permutation of the axes and with a mirror (to summation order)."""
    ph = I.PAPER_PHYS
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v)
    C = LATTICES[q]
    rho = droplet3(10, 3.0, ph, noise=1e-2, seed=3)
    f = orc.step3(scheme, p, orc.init3(scheme, p, rho, q=q), 15)
    sh = (3, -4, 5)
    g = orc.step3(scheme, p, orc.init3(scheme, p, np.roll(rho, sh, axis=(0, 1, 2)), q=q), 15)
    assert np.array_equal(np.roll(f, sh, axis=(0, 1, 2)), g)
    # array axes are (z, y, x); new field(x', y', z') = old(x, y, z) with
    # (x', y', z') = (y, z, x): new[z', y', x'] = old[z, y, x] -> transpose
    # cyclic permutation: the new field at (x', y', z') = (y, z, x) is the old
    # one at (x, y, z); arrays are indexed [z, y, x]
    perm = _index_map(C, lambda c: np.array([c[1], c[2], c[0]]))
    z, y, x = np.mgrid[0:10, 0:10, 0:10]
    rho_p = np.empty_like(rho)
    rho_p[x, z, y] = rho[z, y, x]
    g = orc.step3(scheme, p, orc.init3(scheme, p, rho_p, q=q), 15)
    f_p = np.empty_like(f)
    f_p[x, z, y] = f[z, y, x][..., np.argsort(perm)]
    np.testing.assert_allclose(g, f_p, rtol=0, atol=1e-13)
    mir = _index_map(C, lambda c: np.array([-c[0], c[1], c[2]]))
    rho_m = np.roll(rho[:, :, ::-1], 1, axis=2)
    g = orc.step3(scheme, p, orc.init3(scheme, p, rho_m, q=q), 15)
    f_m = np.roll(f[:, :, ::-1, :], 1, axis=2)[..., mir]
    np.testing.assert_allclose(g, f_m, rtol=0, atol=1e-13)


@pytest.mark.parametrize("scheme", STEP_SCHEMES)
def test_shear_wave_viscosity3(orc, scheme, q):
    """A small shear wave u_x(z) = U sin(k z) decays as exp(-nu k^2 t) with
    nu = cs2 (tau - 1/2) (no free energy: beta = kappa = 0)."""
    tau, n = 0.9, 32
    p = orc.Params(tau, 0.0, 0.0, 1.0, 0.1)
    k = 2 * np.pi / n
    z = np.arange(n)[:, None, None] * np.ones((1, 2, 2))
    ux = 1e-3 * np.sin(k * z)
    f = orc.init3(scheme, p, np.ones((n, 2, 2)), (ux, np.zeros_like(ux), np.zeros_like(ux)), q=q)

    def amp(f):
        return 2 * np.mean(orc.macro3(scheme, p, f)["ux"] * np.sin(k * z))

    f = orc.step3(scheme, p, f, 100)
    a1 = amp(f)
    f = orc.step3(scheme, p, f, 1000)
    a2 = amp(f)
    nu = -np.log(a2 / a1) / (1000 * k * k)
    assert abs(nu / (CS2 * (tau - 0.5)) - 1) < 0.01


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_wb_flat_interface_fixed_point3(orc, axis, q):
    """Sec. III in 3-D: the discrete equilibrium of a flat interface (mu =
    const, solved independently) is an exact fixed point of the WB step
    whichever axis it varies along, and not one of the standard step."""
    ph = I.PAPER_PHYS
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v)
    n = 41
    W = orc.equilibrium_width(p)
    guess = I.tanh_slab(n, p.rho_l, p.rho_v, 10.5, 29.5, W)
    prof, _ = flat_equilibrium(p.beta, p.kappa, p.rho_l, p.rho_v, n, guess.sum(), guess)
    shape = [3, 3, 3]
    shape[axis] = n
    rho = np.broadcast_to(prof.reshape([-1 if a == axis else 1 for a in range(3)]), shape).copy()
    f = orc.init3("well_balanced", p, rho, q=q)
    g = orc.step3("well_balanced", p, f, 100)
    assert np.abs(g - f).max() < 1e-13
    assert orc.observe3("well_balanced", p, g)["max_u"] < 1e-14
    fs = orc.init3("standard", p, rho, q=q)
    gs = orc.step3("standard", p, fs, 5)
    assert orc.observe3("standard", p, gs)["max_u"] > 1e-6
