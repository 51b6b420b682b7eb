"""The seeded input generators (shared by the oracle and the GPU tests): SU(3) links,
APE smearing, sources, and the device-side link generator against the host one."""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def _su3_defect(U):
    U = U.reshape(-1, 3, 3)
    unit = np.abs(np.einsum("nij,nkj->nik", U, U.conj()) - np.eye(3)).max()
    det = np.abs(np.linalg.det(U) - 1).max()
    return unit, det


def test_random_and_smeared_links_are_su3():
    L = (4, 4, 4, 6)
    for U in (synth.random_links(L, 0.7, 3), synth.smeared_links(L, 0.7, 3, 0.6, 3)):
        assert U.shape == (4, 384, 3, 3)
        unit, det = _su3_defect(U)
        assert unit < 1e-13 and det < 1e-13
    assert _su3_defect(synth.unit_links(L)) == (0.0, 0.0)


def test_seeds_reproduce_and_differ():
    L = (4, 4, 4, 4)
    assert np.array_equal(synth.random_links(L, 0.5, 11), synth.random_links(L, 0.5, 11))
    assert not np.array_equal(synth.random_links(L, 0.5, 11), synth.random_links(L, 0.5, 12))


def test_smearing_smooths_the_field():
    """APE smearing raises the average plaquette (the field gets closer to unit links)."""
    L = (4, 4, 4, 4)

    def plaq(U):
        V = 256
        tot = 0.0
        for mu in range(4):
            for nu in range(mu + 1, 4):
                Umu_xnu = synth._shift(U[mu], L, nu, +1)
                Unu_xmu = synth._shift(U[nu], L, mu, +1)
                P = U[mu] @ Unu_xmu @ Umu_xnu.conj().transpose(0, 2, 1) @ U[nu].conj().transpose(0, 2, 1)
                tot += np.trace(P, axis1=1, axis2=2).real.sum() / 3
        return tot / (6 * V)

    U = synth.random_links(L, 0.7, 5)
    S = synth.ape_smear(U, L, 0.6, 3)
    assert plaq(S) > plaq(U) + 0.05
    assert np.allclose(synth.ape_smear(U, L, 0.0, 2), U, atol=1e-13)


def test_device_generator_matches_host():
    L = (4, 4, 4, 4)
    host = synth.smeared_links(L, 0.5, 1703, 0.6, 3)
    dev = synth.smeared_links_torch(L, 0.5, 1703, 0.6, 3, device="cpu").numpy()
    assert np.abs(dev - host).max() < 1e-12


def test_sources():
    L = (4, 4, 4, 4)
    p = synth.point_sources_12(L)
    assert p.shape == (12, 256, 4, 3)
    assert np.array_equal(p[:, 0].reshape(12, 12), np.eye(12))
    assert np.abs(p[:, 1:]).max() == 0
    g = synth.gaussian_source(L, 7, nrhs=2)
    assert np.allclose(np.linalg.norm(g.reshape(2, -1), axis=1), 1.0)
