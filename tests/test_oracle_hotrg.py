"""Pins of the oracle's HOTRG loop.

Each pin compares the oracle with something other than itself:
brute-force contraction of small tori (transfer matrices, direct network
sums), Onsager's exact free energy together with the accuracy the paper
prints for this method, closed-form limits, and invariances.  The last
block plants plausible mistakes in the oracle and checks that a pin fails.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.special import iv

from oracle import exact, hotrg, tensors

BETA_C = math.log(1 + math.sqrt(2)) / 2
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
UNTRUNCATED = 10**9


def torus_from_steps(K):
    """Lattice covered after K directional steps: the first step merges
    vertically, the second horizontally, and so on."""
    return 2 ** (K // 2), 2 ** ((K + 1) // 2)


def network_torus(T, Lx, Ly):
    """Z of the network of copies of T on an Lx-by-Ly torus, summed
    directly over every bond index (no coarse-graining)."""
    letters = iter("abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ")
    h = [[next(letters) for _ in range(Ly)] for _ in range(Lx)]
    v = [[next(letters) for _ in range(Ly)] for _ in range(Lx)]
    subs = [h[(x - 1) % Lx][y] + v[x][(y - 1) % Ly] + h[x][y] + v[x][y]
            for y in range(Ly) for x in range(Lx)]
    return np.einsum(",".join(subs) + "->", *([T] * (Lx * Ly)), optimize=False)


def paper_error_law(D):
    """|df/f| at Tc predicted from the paper's D = 64 value (1.91e-9) and
    its fitted exponent alpha = 4.12 (Sec. 3.2)."""
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        pv = json.load(f)["ising"]
    e64 = pv["max_rel_error_d64_2p20"]["value"]
    alpha = pv["error_exponent_alpha"]["value"]
    return e64 * (64.0 / D) ** alpha


# ---------------------------------------------------------------- pins ----

def pin_random_torus(seed=3, D=2, K=3):
    """Relative deviation of untruncated HOTRG from the direct torus sum for
    a random non-symmetric positive tensor."""
    T = np.random.default_rng(seed).uniform(0.1, 1.0, (D, D, D, D))
    Lx, Ly = torus_from_steps(K)
    want = math.log(network_torus(T, Lx, Ly)) / (Lx * Ly)
    got = hotrg.run(T, UNTRUNCATED, K).lnz_per_site
    return abs(got - want) / abs(want)


def pin_ising_torus(beta=BETA_C, K=4):
    Lx, Ly = torus_from_steps(K)
    want = exact.ising_torus(beta, Lx, Ly)
    got = hotrg.run(tensors.ising(beta), UNTRUNCATED, K).lnz_per_site
    return abs(got - want) / abs(want)


def pin_truncated_tc(D, K=40):
    """Ratio of the oracle's |df/f| at Tc to the paper's error law."""
    got = hotrg.run(tensors.ising(BETA_C), D, K).lnz_per_site
    err = abs(got - exact.onsager_tc()) / exact.onsager_tc()
    return err / paper_error_law(D)


# --------------------------------------------------- pairwise contractions --

def test_environment_matches_nested_loops():
    # M[(i,j),(k,l)] = sum T[j,a,b,e] T[i,e,c,d] T[l,a,b,f] T[k,f,c,d]  (Sec. 2)
    rng = np.random.default_rng(0)
    dx, dy = 2, 3
    T = rng.standard_normal((dx, dy, dx, dy))
    M = hotrg.environment(T).reshape(dx, dx, dx, dx)
    for i, j, k, l in itertools.product(range(dx), repeat=4):
        s = 0.0
        for a, e, f, d in itertools.product(range(dy), repeat=4):
            for b, c in itertools.product(range(dx), repeat=2):
                s += T[j, a, b, e] * T[i, e, c, d] * T[l, a, b, f] * T[k, f, c, d]
        assert M[i, j, k, l] == pytest.approx(s, rel=1e-12, abs=1e-12)


def test_coarse_tensor_matches_nested_loops():
    # T~[i,j,k,l] = sum U[a,b,i] T[b,j,d,c] T[a,c,e,l] U[e,d,k]  (Sec. 2)
    rng = np.random.default_rng(1)
    dx, dy, dn = 2, 3, 3
    T = rng.standard_normal((dx, dy, dx, dy))
    U = rng.standard_normal((dx, dx, dn))
    Tt = hotrg.coarse_tensor(T, U)
    assert Tt.shape == (dn, dy, dn, dy)
    for i, j, k, l in itertools.product(range(dn), range(dy), range(dn), range(dy)):
        s = 0.0
        for a, b, d, e in itertools.product(range(dx), repeat=4):
            for c in range(dy):
                s += U[a, b, i] * T[b, j, d, c] * T[a, c, e, l] * U[e, d, k]
        assert Tt[i, j, k, l] == pytest.approx(s, rel=1e-12, abs=1e-12)


def test_environment_is_symmetric_psd_and_svd_equals_eigh():
    T = hotrg.rotate(np.random.default_rng(2).standard_normal((3, 4, 3, 4)))
    M = hotrg.environment(T)
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    w = np.linalg.eigvalsh(M)[::-1]
    assert w[-1] >= -1e-13 * w[0]
    _, s, _, _ = hotrg.projector(M, 4)
    assert np.abs(s - w).max() <= 1e-13 * w[0]


# ---------------------------------------------- exact untruncated results --

@pytest.mark.parametrize("beta", [0.3, BETA_C, 0.6])
@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
def test_untruncated_ising_equals_transfer_matrix(beta, K):
    assert pin_ising_torus(beta, K) <= 1e-13


@pytest.mark.parametrize("seed,D,K", [(3, 2, 1), (3, 2, 2), (3, 2, 3), (4, 3, 1), (4, 3, 2), (5, 2, 3)])
def test_untruncated_random_tensor_equals_direct_sum(seed, D, K):
    assert pin_random_torus(seed, D, K) <= 1e-13


def test_untruncated_xy_equals_angle_quadrature():
    # one vertical step = the 1x2 torus; n_max = 8 leaves a character tail
    # of about I_9(0.5)/I_0(0.5) ~ 1e-11
    beta = 0.5
    got = hotrg.run(tensors.xy(beta, 8), UNTRUNCATED, 1).lnz_per_site
    assert got == pytest.approx(exact.xy_torus(beta, 1, 2), rel=1e-10)


def test_untruncated_xy_two_steps_equals_direct_sum():
    T = tensors.xy(0.7, 2)
    got = hotrg.run(T, UNTRUNCATED, 2).lnz_per_site
    want = math.log(network_torus(T, 2, 2)) / 4
    assert got == pytest.approx(want, rel=1e-13)


def test_scale_of_initial_tensor_shifts_lnz_exactly():
    T = tensors.ising(0.4)
    a = hotrg.run(T, 8, 12).lnz_per_site
    b = hotrg.run(3.7 * T, 8, 12).lnz_per_site
    assert b - a == pytest.approx(math.log(3.7), rel=1e-12)


# -------------------------------------------------- truncated, large lattice --

@pytest.mark.parametrize("D", [8, 16])
def test_truncated_error_follows_paper_law(D):
    # the paper prints 1.91e-9 at D = 64 and |df/f| ~ D^-4.12 (Sec. 3.2);
    # the law extrapolated to small D must hold within a factor of 2
    r = pin_truncated_tc(D)
    assert 0.5 <= r <= 2.0, r


@pytest.mark.slow
def test_truncated_d32_and_exponent():
    # D = 32 over 2^15 x 2^15 sites: within 1.5x of the paper's law, and the
    # exponent between D = 16 and 32 close to the paper's 4.12
    g = hotrg.run(tensors.ising(BETA_C), 32, 30).lnz_per_site
    e32 = abs(g - exact.onsager_tc()) / exact.onsager_tc()
    assert 1 / 1.5 <= e32 / paper_error_law(32) <= 1.5
    g16 = hotrg.run(tensors.ising(BETA_C), 16, 40).lnz_per_site
    e16 = abs(g16 - exact.onsager_tc()) / exact.onsager_tc()
    alpha = math.log(e16 / e32) / math.log(2.0)
    assert 3.8 <= alpha <= 4.5


def test_error_is_largest_at_tc():
    # Sec. 3.2: the largest deviation is at Tc
    errs = {}
    for T in (2.0, exact.TC_ISING, 2.5):
        g = hotrg.run(tensors.ising(1.0 / T), 16, 40).lnz_per_site
        errs[T] = abs(g - exact.onsager_hyper(1.0 / T))
    assert errs[exact.TC_ISING] > 10 * max(errs[2.0], errs[2.5])


def test_potts_q2_is_ising_at_half_beta():
    # W_Potts(q=2, beta) = e^(beta/2) W_Ising(beta/2): ln Z/N differs by beta
    # (two bonds per site); the tensors differ by an orthogonal leg gauge
    beta = 0.9
    p = hotrg.run(tensors.potts(beta, 2), 16, 24).lnz_per_site
    i = hotrg.run(tensors.ising(beta / 2), 16, 24).lnz_per_site
    assert p - i == pytest.approx(beta, rel=1e-12)


def test_xy_high_temperature_series():
    beta = 0.1
    series, t = exact.xy_high_temperature(beta)
    g = hotrg.run(tensors.xy(beta, 3), 16, 20).lnz_per_site
    assert abs(g - series) <= 10 * t**6
    assert abs(g - 2 * math.log(iv(0, beta))) > t**4  # the t^4 term is seen


def test_orthogonal_gauge_invariance():
    # T'[l,u,r,d] = O1[l,l'] O2[u,u'] O1[r,r'] O2[d,d'] T[l',u',r',d'] is the
    # same network; ln Z/N and spectra must not change (truncated run)
    rng = np.random.default_rng(7)
    T = tensors.ising(0.42)
    T = T + 0.05 * rng.uniform(0, 1, T.shape)  # break the leg symmetry
    O1, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    O2, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    Tg = np.einsum("La,Ub,Rc,Dd,abcd->LURD", O1, O2, O1, O2, T)
    a = hotrg.run(T, 8, 16, spec_len=9)
    b = hotrg.run(Tg, 8, 16, spec_len=9)
    assert b.lnz_per_site == pytest.approx(a.lnz_per_site, rel=1e-12)
    for sa, sb in zip(a.spectra, b.spectra):
        assert np.abs(sa - sb).max() <= 1e-12


def test_multiplet_rule_drops_whole_cluster():
    # XY spectra have exact pairs (charge +-n); the multiplet rule must not
    # keep one member of a pair
    T = tensors.xy(1.0, 3)
    M = hotrg.environment(T)
    _, s, _, _ = hotrg.projector(M, 49)
    for d_cut in range(2, 30):
        U, s, d_new, kept = hotrg.projector(M, d_cut, "multiplet", 1e-10)
        assert kept <= d_new
        if kept < s.size:
            assert s[kept - 1] - s[kept] > 1e-10 * s[0]
        assert np.all(U[:, kept:] == 0.0)


def test_dims_schedule_matches_run():
    res = hotrg.run(tensors.ising(0.4), 8, 7)
    got = [(s.dx, s.dy, s.d_new) for s in res.steps]
    assert got == hotrg.dims_schedule(2, 8, 7)
    assert got[:4] == [(2, 2, 4), (2, 4, 4), (4, 4, 8), (4, 8, 8)]


# ------------------------------------------------------ planted mistakes --

def _coarse_tensor_transposed_U(T, U3):
    X1 = np.tensordot(U3, T, axes=([1], [0]))
    X2 = np.tensordot(X1, T, axes=([0, 4], [0, 1]))
    Tt = np.tensordot(X2, U3, axes=([2, 3], [0, 1]))  # U[d,e,k] instead of U[e,d,k]
    return Tt.transpose(0, 1, 3, 2)


def _environment_wrong_pairing(T):
    dx = T.shape[0]
    A = np.tensordot(T, T, axes=([1, 2], [1, 2]))
    B = np.tensordot(T, T, axes=([2, 3], [2, 3]))
    M = np.tensordot(B, A, axes=([1, 3], [3, 1]))  # e paired with f
    return M.transpose(0, 2, 1, 3).reshape(dx * dx, dx * dx)


def _projector_smallest(M, d_cut, trunc="plain", tau=1e-10):
    U, s, d_new, kept = _PROJECTOR(M, d_cut, trunc, tau)
    Uf, _, _ = np.linalg.svd(M)
    return Uf[:, ::-1][:, :d_new].copy(), s, d_new, kept


def _rotate_missing(T):
    return T  # the orthogonal direction is never coarse-grained


_PROJECTOR = hotrg.projector


def test_planted_transposed_projector_is_caught(monkeypatch):
    monkeypatch.setattr(hotrg, "coarse_tensor", _coarse_tensor_transposed_U)
    assert pin_random_torus() > 1e-6


def test_planted_wrong_environment_is_caught(monkeypatch):
    monkeypatch.setattr(hotrg, "environment", _environment_wrong_pairing)
    assert pin_truncated_tc(16) > 10.0


def test_planted_smallest_vectors_is_caught(monkeypatch):
    monkeypatch.setattr(hotrg, "projector", _projector_smallest)
    assert pin_truncated_tc(8, K=20) > 10.0


def test_planted_missing_rotation_is_caught(monkeypatch):
    monkeypatch.setattr(hotrg, "rotate", _rotate_missing)
    assert pin_random_torus(D=2, K=2) > 1e-6


def test_coarse_tensor_slice_matches_full():
    rng = np.random.default_rng(11)
    T = rng.standard_normal((3, 4, 3, 4))
    U = rng.standard_normal((3, 3, 5))
    full = hotrg.coarse_tensor(T, U)
    for i, k in [(0, 0), (2, 4), (4, 1)]:
        assert np.abs(hotrg.coarse_tensor_slice(T, U, i, k) - full[i, :, k, :]).max() <= 1e-12


def test_gxy_nematic_limit_is_xy():
    # Delta = 0: the weight depends on 2(theta_i - theta_j) only, so theta -> 2 theta maps
    # the model onto XY at the same beta; in the tensor network the odd charges carry
    # zero weight and the even ones are the XY tensor (n_max = 2m against m)
    a = hotrg.run(tensors.gxy(1.0, 0.0, 4), 10, 8, trunc="multiplet", tau=1e-10)
    b = hotrg.run(tensors.xy(1.0, 2), 10, 8, trunc="multiplet", tau=1e-10)
    assert a.lnz_per_site == pytest.approx(b.lnz_per_site, rel=1e-12)


def test_gxy_untruncated_one_step_equals_charge_sum_and_quadrature():
    # 1x2 torus (one vertical step, untruncated).  Charge conservation at a
    # site forces the two vertical bonds to carry the same charge, so
    # Z = (sum_n c_n)^2 * sum_n c_n^2 over the kept charges; with many charges
    # the same sum is the angle integral of the four bond weights.  The
    # nematic coefficients fall off only like (beta(1-delta)/2)^(n/2) / (n/2)!,
    # so the quadrature comparison uses n_max = 40 on the weights alone.
    beta, delta = 0.9, 0.5
    c = tensors.gxy_weights(beta, delta, 3)
    r = hotrg.run(tensors.gxy(beta, delta, 3), UNTRUNCATED, 1)
    assert r.lnz_per_site == pytest.approx(np.log(c.sum() ** 2 * (c * c).sum()) / 2, rel=1e-13)
    c = tensors.gxy_weights(beta, delta, 40)
    N = 96
    th = 2 * np.pi * np.arange(N) / N
    w = np.exp(beta * delta * np.cos(th) + beta * (1 - delta) * np.cos(2 * th))
    Z = np.mean(w * w) * np.exp(2 * beta)  # two vertical bonds, two self-bonds at angle 0
    assert c.sum() ** 2 * (c * c).sum() == pytest.approx(Z, rel=1e-13)


# ------------------------------------------------------ truncation error --
# epsilon = 1 - sum_{m <= kept} s_m / sum_m s_m is the share of the
# environment's trace that the projector does not keep (M is PSD, so its
# singular values are its eigenvalues and sum to trace(M)).  Pinned without
# the function's own formula: a known spectrum in closed form, and the trace
# of M projected onto the kept columns, 1 - trace(U U^T M) / trace(M).


def _pin_truncation_error():
    worst = 0.0
    # closed form: M = Q diag(8, 4, 2, 1, 1/2) Q^T, Q a random rotation
    lam = np.array([8.0, 4.0, 2.0, 1.0, 0.5])
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((5, 5)))
    M = Q @ np.diag(lam) @ Q.T
    for d_cut, want in [(1, 1.0 - 8.0 / 15.5), (2, 1.0 - 12.0 / 15.5), (3, 1.0 - 14.0 / 15.5),
                        (4, 1.0 - 15.0 / 15.5), (5, 0.0)]:
        _, s, _, kept = hotrg.projector(M, d_cut)
        worst = max(worst, abs(hotrg.truncation_error(s, kept) - want))
    # projected trace of real environments (plain and multiplet cuts)
    for T, d_cut, trunc in [(tensors.ising(0.44), 3, "plain"), (tensors.xy(1.0, 2), 7, "multiplet"),
                            (tensors.potts(0.9, 3), 4, "plain")]:
        M = hotrg.environment(T)
        U, s, _, kept = hotrg.projector(M, d_cut, trunc, 1e-10)
        direct = 1.0 - np.trace(U @ U.T @ M) / np.trace(M)
        worst = max(worst, abs(hotrg.truncation_error(s, kept) - direct))
    return worst


def test_truncation_error_pinned():
    assert _pin_truncation_error() <= 1e-13


@pytest.mark.parametrize("wrong", [
    lambda s, kept: float(1.0 - (s[:kept] ** 2).sum() / (s ** 2).sum()),  # squared values
    lambda s, kept: float(1.0 - s[:kept].sum() / s[0]),                 # divided by s_1
    lambda s, kept: float(1.0 - s[:kept + 1].sum() / s.sum()),          # one value too many
])
def test_planted_truncation_error_is_caught(monkeypatch, wrong):
    monkeypatch.setattr(hotrg, "truncation_error", wrong)
    assert _pin_truncation_error() > 1e-3
