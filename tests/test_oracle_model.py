"""Oracle pins: the lattice-summed dipole kernel, the field and the energy.

Each check below compares the oracle against something other than itself:
closed forms (image sums over integer lattices, the Z^2 lattice sum
4 zeta(3/2) beta(3/2)), symmetries of the dipole tensor, an independent
literal evaluation of eq. (1) with explicit periodic images (Sec. 2.1), and
the full-energy difference for the single-site move.
"""
import numpy as np
import pytest
from scipy import special

from paper_1211_6234_amd import workloads


# ----------------------------------------------------------------- helpers
def box_weight(c, L, M):
    """Edge weight of an integer image coordinate in |c| <= (M + 1/2) L."""
    twice = 2 * np.abs(c)
    edge = (2 * M + 1) * L
    return np.where(twice < edge, 1.0, np.where(twice == edge, 0.5, 0.0))


def box_inverse_cube_sum(L, M):
    """sum over integer r != 0 in the box, weighted, of |r|^-3 (independent of W)."""
    R = (M + 1) * L
    c = np.arange(-R, R + 1)
    X, Y = np.meshgrid(c, c, indexing="xy")
    w = box_weight(X, L, M) * box_weight(Y, L, M)
    r2 = (X * X + Y * Y).astype(np.float64)
    r2[R, R] = 1.0
    w[R, R] = 0.0
    return float(np.sum(w / r2 ** 1.5))


def brute_dipole_energy(L, M, s, g):
    """Literal eq. (1): (g/2) sum_n sum_m sum_images w (s_n.s_m - 3 s_n.r^ s_m.r^)/r^3."""
    N = L * L
    xs, ys = np.arange(N) % L, np.arange(N) // L
    S = s.T  # [N][3]
    e = 0.0
    for n in range(N):
        for m in range(N):
            for b in range(-M - 1, M + 2):
                for a in range(-M - 1, M + 2):
                    rx = xs[m] - xs[n] + a * L
                    ry = ys[m] - ys[n] + b * L
                    w = box_weight(rx, L, M) * box_weight(ry, L, M)
                    if w == 0 or (rx == 0 and ry == 0):
                        continue
                    r = np.array([rx, ry, 0.0])
                    d = np.linalg.norm(r)
                    rh = r / d
                    e += w * (S[n] @ S[m] - 3.0 * (S[n] @ rh) * (S[m] @ rh)) / d ** 3
    return 0.5 * g * e


def random_spins(L, seed):
    return workloads.random_spins(L * L, 1, seed)[0].astype(np.float64)


# ----------------------------------------------------------------- the kernel W
@pytest.mark.parametrize("L,M", [(8, 3), (16, 8), (5, 2), (2, 4)])
def test_self_image_term_closed_form(orc, L, M):
    W = orc.lattice_sum_kernel(L, M)
    a = np.arange(-M, M + 1)
    A, B = np.meshgrid(a, a)
    q = (A * A + B * B).astype(np.float64)
    q[M, M] = np.inf
    S_M = float(np.sum(q ** -1.5))
    expect = S_M / L ** 3 * np.array([-0.5, -0.5, 0.0, 1.0])
    got = W[:, 0, 0]
    assert np.allclose(got, expect, rtol=1e-13, atol=1e-15 * S_M / L ** 3)


@pytest.mark.parametrize("L,M", [(8, 3), (12, 2), (7, 1), (16, 0)])
def test_kernel_symmetries(orc, L, M):
    W = orc.lattice_sum_kernel(L, M)
    scale = np.abs(W).max()
    tol = 1e-14 * scale
    idx = (-np.arange(L)) % L
    # trace-free: Wxx + Wyy + Wzz = 0 (in-plane separations)
    assert np.abs(W[0] + W[1] + W[3]).max() < tol
    # even: W(rho) = W(-rho)
    for c in range(4):
        assert np.abs(W[c] - W[c][idx][:, idx]).max() < tol
    # x <-> y mirror swaps xx and yy (arrays are [y][x])
    assert np.abs(W[0] - W[1].T).max() < tol
    assert np.abs(W[2] - W[2].T).max() < tol
    # xy is odd in each coordinate separately
    assert np.abs(W[2] + W[2][:, idx]).max() < tol
    assert np.abs(W[2] + W[2][idx, :]).max() < tol
    assert abs(W[2].sum()) < L * L * tol


@pytest.mark.parametrize("L,M", [(16, 8), (8, 3), (6, 0)])
def test_uniform_state_dipole_energy(orc, L, M):
    """Uniform state n: E_dip/N = (g/2) S_box (3 n_z^2 - 1)/2 with S_box an
    independent weighted box sum of |r|^-3 over integer vectors."""
    g = 0.7
    Sb = box_inverse_cube_sum(L, M)
    W = orc.lattice_sum_kernel(L, M)
    N = L * L
    p = orc.params(T=1.0, J=0.0, g=g)
    rng = np.random.default_rng(3)
    dirs = [np.array([0, 0, 1.0]), np.array([1.0, 0, 0]), np.array([0, 1.0, 0])]
    dirs += [v / np.linalg.norm(v) for v in rng.normal(size=(3, 3))]
    for n in dirs:
        s = np.repeat(n[:, None], N, axis=1)
        e = orc.energy(L, W, p, s)["dip"] / N
        expect = 0.5 * g * Sb * (3 * n[2] ** 2 - 1) / 2
        assert abs(e - expect) <= 1e-12 * abs(0.5 * g * Sb), (n, e, expect)


def test_box_sum_converges_to_lattice_zeta():
    """sum over Z^2 \\ {0} of |r|^-3 = 4 zeta(3/2) beta(3/2); the box misses
    approximately the continuum tail 4 sqrt(2) / a outside half-width a."""
    beta = 4.0 ** -1.5 * (special.zeta(1.5, 0.25) - special.zeta(1.5, 0.75))
    S_inf = 4.0 * special.zeta(1.5) * beta
    assert abs(S_inf - 9.0336216831) < 1e-9
    for L, M in [(16, 8), (32, 8), (64, 4)]:
        a = (M + 0.5) * L
        tail = S_inf - box_inverse_cube_sum(L, M)
        assert abs(tail - 4 * np.sqrt(2) / a) < 0.02 * 4 * np.sqrt(2) / a, (L, M, tail)


def test_kernel_image_tail(orc):
    """Growing the box from half-width a1 to a2 adds to W_zz(rho) the images of
    one site (density 1/L^2) between the two squares: 4 sqrt(2)/L^2 (1/a1 - 1/a2)
    in the continuum limit, and half of that (negated) to W_xx and W_yy."""
    L = 8
    W4, W16 = orc.lattice_sum_kernel(L, 4), orc.lattice_sum_kernel(L, 16)
    a1, a2 = 4.5 * L, 16.5 * L
    add = 4 * np.sqrt(2) / L ** 2 * (1 / a1 - 1 / a2)
    d = W16 - W4
    assert np.abs(d[3] - add).max() < 0.02 * add
    assert np.abs(d[0] + add / 2).max() < 0.03 * add
    assert np.abs(d[1] + add / 2).max() < 0.03 * add


# ------------------------------------------------- all images (Ewald-Harris split)
def _lattice_zeta():
    beta = 4.0 ** -1.5 * (special.zeta(1.5, 0.25) - special.zeta(1.5, 0.75))
    return 4.0 * special.zeta(1.5) * beta


@pytest.mark.parametrize("L", [2, 5, 16])
def test_all_images_independent_of_split(orc, L):
    """The real-space / reciprocal split of Sec. 2.1 is exact: the sum does not
    depend on the splitting length eta (a dropped self term, a wrong factor in
    either part or a wrong sign between them makes it eta-dependent)."""
    ref = orc.lattice_sum_ewald(L, L / 4.0)
    for eta in (L / 9.0, L / 2.5, 0.9 * L):
        W = orc.lattice_sum_ewald(L, eta)
        assert np.abs(W - ref).max() <= 1e-13 * np.abs(ref).max(), eta


@pytest.mark.parametrize("L", [1, 3, 8, 32])
def test_all_images_self_term_closed_form(orc, L):
    """W_inf(0) = (S/L^3) diag(-1/2, -1/2, 1) with S = 4 zeta(3/2) beta(3/2), the
    lattice sum of |r|^-3 over Z^2 minus the origin (Hurwitz zeta, scipy)."""
    W = orc.lattice_sum_ewald(L)
    S = _lattice_zeta()
    for c, want in ((0, -0.5 * S), (1, -0.5 * S), (2, 0.0), (3, S)):
        assert abs(W[c, 0, 0] * L ** 3 - want) <= 1e-13 * S, (c, W[c, 0, 0] * L ** 3, want)


def test_all_images_is_the_limit_of_the_box_sums(orc):
    """W_inf - W_M is what the box of half-width a = (M + 1/2) L misses: in the
    continuum limit 4 sqrt(2)/(L^2 a) on zz and half of it, negated, on xx and
    yy, 0 on xy; the mismatch falls like 1/M^2."""
    L = 8
    Winf = orc.lattice_sum_ewald(L)
    errs = []
    for M in (12, 24):
        a = (M + 0.5) * L
        miss = 4 * np.sqrt(2) / (L ** 2 * a)
        d = Winf - orc.lattice_sum_kernel(L, M)
        err = max(np.abs(d[3] - miss).max(), np.abs(d[0] + miss / 2).max(), np.abs(d[1] + miss / 2).max(),
                  np.abs(d[2]).max())
        assert err < 0.01 * miss, (M, err, miss)
        errs.append(err / miss)
    assert errs[1] < errs[0] / 3.0


def test_all_images_symmetries(orc):
    """Even in rho, trace-free, xy odd under x -> -x, xx <-> yy under x <-> y."""
    L = 12
    W = orc.lattice_sum_ewald(L)
    neg = lambda A: np.roll(np.roll(A[::-1, ::-1], 1, 0), 1, 1)
    for c in range(4):
        assert np.abs(W[c] - neg(W[c])).max() <= 1e-14 * np.abs(W).max()
    assert np.abs(W[0] + W[1] + W[3]).max() <= 1e-14 * np.abs(W).max()
    mx = lambda A: np.roll(A[:, ::-1], 1, 1)
    assert np.abs(W[2] + mx(W[2])).max() <= 1e-14 * np.abs(W).max()
    assert np.abs(W[0] - W[1].T).max() <= 1e-14 * np.abs(W).max()


# ----------------------------------------------------------------- the field
@pytest.mark.parametrize("L,M", [(4, 2), (6, 1), (3, 2), (2, 3)])
def test_field_table_vs_table_free(orc, L, M):
    s = random_spins(L, 10 + L)
    W = orc.lattice_sum_kernel(L, M)
    h = orc.field(L, W, s)
    hi = orc.field_images(L, M, s)
    assert np.abs(h - hi).max() < 1e-13 * np.abs(hi).max()


@pytest.mark.parametrize("L,M", [(2, 2), (3, 1), (4, 1)])
def test_energy_vs_literal_eq1(orc, L, M):
    g = 0.37
    s = random_spins(L, 20 + L)
    W = orc.lattice_sum_kernel(L, M)
    p = orc.params(T=1.0, J=0.0, g=g)
    e = orc.energy(L, W, p, s)["dip"]
    ref = brute_dipole_energy(L, M, s, g)
    assert abs(e - ref) < 1e-12 * max(1.0, abs(ref))


def test_field_impulse_response(orc):
    L, M = 8, 2
    W = orc.lattice_sum_kernel(L, M)
    N = L * L
    for a in range(3):
        s = np.zeros((3, N))
        s[a, 0] = 1.0
        h = orc.field(L, W, s).reshape(3, L, L)
        if a == 0:
            exp = np.stack([W[0], W[2], 0 * W[0]])
        elif a == 1:
            exp = np.stack([W[2], W[1], 0 * W[0]])
        else:
            exp = np.stack([0 * W[0], 0 * W[0], W[3]])
        assert np.abs(h - exp).max() < 1e-15


def test_field_covariances(orc):
    L, M = 8, 3
    W = orc.lattice_sum_kernel(L, M)
    s = random_spins(L, 7).reshape(3, L, L)
    h = orc.field(L, W, s.reshape(3, -1)).reshape(3, L, L)
    tol = 1e-13 * np.abs(h).max()
    # translation
    st = np.roll(s, (3, 5), axis=(1, 2))
    ht = orc.field(L, W, st.reshape(3, -1)).reshape(3, L, L)
    assert np.abs(ht - np.roll(h, (3, 5), axis=(1, 2))).max() < tol
    # linearity and time reversal
    s2 = random_spins(L, 8).reshape(3, L, L)
    h2 = orc.field(L, W, s2.reshape(3, -1)).reshape(3, L, L)
    hl = orc.field(L, W, (2.0 * s - 0.5 * s2).reshape(3, -1)).reshape(3, L, L)
    assert np.abs(hl - (2.0 * h - 0.5 * h2)).max() < 4 * tol
    # 90 degree rotation: site (x, y) -> (-y, x), spin (sx, sy) -> (-sy, sx)
    def rot(v):
        out = np.empty_like(v)
        for y in range(L):
            for x in range(L):
                out[:, x % L, (-y) % L] = [-v[1, y, x], v[0, y, x], v[2, y, x]]
        return out
    hr = orc.field(L, W, rot(s).reshape(3, -1)).reshape(3, L, L)
    assert np.abs(hr - rot(h)).max() < tol
    # mirror x -> -x with sx -> -sx
    def mir(v):
        out = v[:, :, (-np.arange(L)) % L].copy()
        out[0] *= -1
        return out
    hm = orc.field(L, W, mir(s).reshape(3, -1)).reshape(3, L, L)
    assert np.abs(hm - mir(h)).max() < tol


# ----------------------------------------------------------------- energies and dE
@pytest.mark.parametrize("L,M", [(2, 2), (4, 1), (5, 2), (8, 3)])
def test_delta_e_equals_full_energy_difference(orc, L, M):
    W = orc.lattice_sum_kernel(L, M)
    rng = np.random.default_rng(L)
    for trial in range(6):
        p = orc.params(T=1.0, J=rng.uniform(-1, 2), K2=rng.uniform(-2, 2),
                       K4=rng.uniform(-1, 1), g=rng.uniform(0, 0.5))
        s = random_spins(L, 100 * L + trial)
        h = orc.field(L, W, s)
        k = int(rng.integers(L * L))
        S = rng.normal(size=3)
        S /= np.linalg.norm(S)
        dE = orc.delta_e(L, W, p, s, h, k, S)
        s2 = s.copy()
        s2[:, k] = S
        e1, e0 = orc.energy(L, W, p, s2), orc.energy(L, W, p, s)
        ref = e1["total"] - e0["total"]
        scale = sum(abs(e1[t]) + abs(e0[t]) for t in ("ex", "dip", "ani")) / (L * L)
        assert abs(dE - ref) < 1e-12 * max(scale, abs(ref)), (dE, ref)


def test_exchange_and_anisotropy_closed_forms(orc):
    for L in (2, 4, 7):
        N = L * L
        W = orc.lattice_sum_kernel(L, 1)
        up = np.zeros((3, N)); up[2] = 1.0
        ex = np.zeros((3, N)); ex[0] = 1.0
        p = orc.params(T=1.0, J=1.3, K2=0.0, K4=0.0, g=0.0)
        assert abs(orc.energy(L, W, p, up)["ex"] / N + 2 * 1.3) < 1e-14
        # paper's anisotropy K((1-a) sz^2 + a sz^4) -> K2 = -K(1-a), K4 = -K a
        for K in (-15.0, -1.0):
            for a in (-1.0, 0.0, 2.0, 0.5):
                K2, K4 = -K * (1 - a), -K * a
                p = orc.params(T=1.0, J=0.0, K2=K2, K4=K4, g=0.0)
                # in-plane minus perpendicular anisotropy energy per spin is -K for every a
                d = (orc.energy(L, W, p, ex)["ani"] - orc.energy(L, W, p, up)["ani"]) / N
                assert abs(d + K) < 1e-12 * abs(K)
                # curvature at the pole: d^2 E_A / d theta^2 = 2 K2 + 4 K4 = -2 K (1 + a)
                hstep = 1e-4
                def ea(th):
                    sv = np.zeros((3, N)); sv[0] = np.sin(th); sv[2] = np.cos(th)
                    return orc.energy(L, W, p, sv)["ani"] / N
                curv = (ea(hstep) - 2 * ea(0.0) + ea(-hstep)) / hstep ** 2
                assert abs(curv - (-2 * K * (1 + a))) < 1e-5 * abs(K) * (1 + abs(a))


def test_interaction_counts_quoted_in_paper():
    """Sec. 2.1: L = 64 needs N = 4096 interactions per spin and C(N, 2),
    over 8e6, per state."""
    N = 64 * 64
    assert N == 4096
    assert N * (N - 1) // 2 == 8386560 > 8e6


def test_paper_stripe_widths_fix_the_exchange_normalisation(orc):
    """Sec. 4.1 states that J/C_D = 8.9 gives a ground state of perpendicular
    stripes of width 8, and the Ising appendix that J/C_D = 1.7 gives the
    thinnest stripes (width 1).  With the pair dipole coupling twice C_D
    relative to the bond exchange, g = 2 / (J/C_D) here, the lowest of the
    stripe energies (all images, L = 64) is at exactly those widths; with
    g = 1 / (J/C_D) it is not (widths 32 and 2).  The scan workload uses
    g = 2 / 8.9."""
    from paper_1211_6234_amd import workloads
    L = 64
    W = orc.lattice_sum_ewald(L)
    widths = (1, 2, 4, 8, 16, 32)

    def best(g):
        e = [orc.energy(L, W, orc.params(T=1.0, J=1.0, g=g), workloads.striped_spins(L, w, 1)[0])["total"]
             for w in widths]
        return widths[int(np.argmin(e))]

    g_scan = workloads.film_scan([1.0])["replicas"][0]["g"]
    assert abs(g_scan - 2 / 8.9) < 1e-15
    assert best(g_scan) == 8 and best(1 / 8.9) == 32
    assert best(2 / 1.7) == 1 and best(1 / 1.7) == 2
