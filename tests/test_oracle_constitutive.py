"""Pins of the oracle's constitutive law against the paper's spatial formulas.

The oracle works in material form (P, A = dP/dF).  These tests re-derive the paper's
Eulerian quantities independently -- Cauchy stress eq. (sig_eq), elasticity tensor
eq. (const_eq) and the tensor D of Sec. 3.1.4 -- and check the push-forward identities,
plus finite differences of the energy and the small-strain (Hooke) limit.
"""
import numpy as np
import pytest


def _rand_F(rng, dim=3, scale=0.25):
    F = np.eye(3)
    F[:dim, :dim] += scale * rng.standard_normal((dim, dim))
    if np.linalg.det(F) <= 0.2:
        F[:dim, :dim] = np.eye(dim) + 0.1 * rng.standard_normal((dim, dim))
    return F


def _paper_sigma(F, mu, lam):
    # eq. (sig_eq): sigma = mu/J (b - I) + lam/J ln J I, b = F F^T
    J = np.linalg.det(F)
    return mu / J * (F @ F.T - np.eye(3)) + lam / J * np.log(J) * np.eye(3)


def _paper_C(F, mu, lam):
    # eq. (const_eq): C_ijkl = lam/J d_ij d_kl + (mu - lam ln J)/J (d_ik d_jl + d_il d_jk)
    J = np.linalg.det(F)
    d = np.eye(3)
    return (lam / J * np.einsum("ij,kl->ijkl", d, d)
            + (mu - lam * np.log(J)) / J * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def _paper_D(F, mu, lam):
    # Sec. 3.1.4: D_ijkl = C_ikjl + d_ij sigma_kl
    C = _paper_C(F, mu, lam)
    s = _paper_sigma(F, mu, lam)
    return np.einsum("ikjl->ijkl", C) + np.einsum("ij,kl->ijkl", np.eye(3), s)


@pytest.mark.parametrize("seed", range(6))
def test_cauchy_stress_is_push_forward_of_P(orc, seed):
    rng = np.random.default_rng(seed)
    F = _rand_F(rng)
    mu, lam = rng.uniform(0.5, 2.0), rng.uniform(0.5, 10.0)
    W, P, A = orc.neo_hooke(F, mu, lam)
    J = np.linalg.det(F)
    np.testing.assert_allclose(P @ F.T / J, _paper_sigma(F, mu, lam), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_material_tangent_is_pull_back_of_spatial_D(orc, seed):
    # A_{iJjL} = J Finv_{Jk} Finv_{Ll} D_{ijkl}: the material tangent equals the paper's D
    # (constitutive + initial-stress parts) pulled back to the reference configuration.
    rng = np.random.default_rng(100 + seed)
    F = _rand_F(rng)
    mu, lam = rng.uniform(0.5, 2.0), rng.uniform(0.5, 10.0)
    _, _, A = orc.neo_hooke(F, mu, lam)
    Fi = np.linalg.inv(F)
    J = np.linalg.det(F)
    A_ref = J * np.einsum("Jk,Ll,ijkl->iJjL", Fi, Fi, _paper_D(F, mu, lam))
    np.testing.assert_allclose(A, A_ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_stress_and_tangent_are_derivatives(orc, seed):
    rng = np.random.default_rng(200 + seed)
    F = _rand_F(rng)
    mu, lam = 1.3, 4.0
    W, P, A = orc.neo_hooke(F, mu, lam)
    h = 1e-6
    Pfd = np.zeros((3, 3)); Afd = np.zeros((3, 3, 3, 3))
    for j in range(3):
        for L in range(3):
            dF = np.zeros((3, 3)); dF[j, L] = h
            Wp, Pp, _ = orc.neo_hooke(F + dF, mu, lam)
            Wm, Pm, _ = orc.neo_hooke(F - dF, mu, lam)
            Pfd[j, L] = (Wp - Wm) / (2 * h)
            Afd[:, :, j, L] = (Pp - Pm) / (2 * h)
    np.testing.assert_allclose(P, Pfd, rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(A, Afd, rtol=1e-6, atol=1e-7)


def test_reference_state_is_hooke(orc):
    mu, lam = 1.0, 10.0
    W, P, A = orc.neo_hooke(np.eye(3), mu, lam)
    d = np.eye(3)
    hooke = lam * np.einsum("iJ,jL->iJjL", d, d) + mu * (np.einsum("ij,JL->iJjL", d, d)
                                                         + np.einsum("iL,Jj->iJjL", d, d))
    assert W == 0.0
    np.testing.assert_array_equal(P, np.zeros((3, 3)))
    np.testing.assert_allclose(A, hooke, atol=1e-15)


def test_energy_closed_form(orc):
    # W = mu/2 (I1 - 3) - mu ln J + lam/2 (ln J)^2 at a diagonal stretch (plane strain: F33 = 1)
    F = np.diag([1.1, 0.9, 1.0])
    mu, lam = 1.0, 10.0
    W, _, _ = orc.neo_hooke(F, mu, lam)
    J = 1.1 * 0.9
    I1 = 1.1 ** 2 + 0.9 ** 2 + 1.0
    assert abs(W - (0.5 * mu * (I1 - 3) - mu * np.log(J) + 0.5 * lam * np.log(J) ** 2)) < 1e-15


def test_inverted_rejected(orc):
    with pytest.raises(ValueError):
        orc.neo_hooke(np.diag([1.0, -0.5, 1.0]), 1.0, 1.0)
