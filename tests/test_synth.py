"""The seeded generators: reproducible streams, SU(3) links, Haar fields."""
import numpy as np

import synth


def test_gauge_field_is_su3_and_chunk_independent():
    L = (4, 4, 2, 6)
    U1 = synth.gauge_field(L, 0.7, seed=3)
    U2 = synth.gauge_field(L, 0.7, seed=3, t_chunk=1)
    assert np.array_equal(U1, U2)
    I = np.eye(3)
    assert np.max(np.abs(U1 @ np.conj(np.swapaxes(U1, -1, -2)) - I)) < 1e-14
    assert np.max(np.abs(np.linalg.det(U1) - 1)) < 1e-14
    # mean-field link: E Re tr U / 3 is about 1 - 2 eps^2 / 3 for small eps
    u0 = np.mean(np.trace(synth.gauge_field((8, 8, 8, 8), 0.3, 0), axis1=-2, axis2=-1).real) / 3
    assert abs(u0 - (1 - 2 * 0.3 ** 2 / 3)) < 0.01
    assert not np.array_equal(U1, synth.gauge_field(L, 0.7, seed=4))


def test_taylor_exponential_equals_eigh_form():
    rng = np.random.default_rng(5)
    A = (rng.standard_normal((2000, 3, 3)) + 1j * rng.standard_normal((2000, 3, 3))) / np.sqrt(2)
    for eps in (0.3, 0.7, 1.0):
        assert np.max(np.abs(synth.exp_i_eps_h(A, eps) - synth.exp_i_eps_h_eigh(A, eps))) < 1e-14


def test_spinors_and_sources():
    L = (2, 2, 2, 4)
    a = synth.gaussian_spinor(L, 1000)
    assert a.shape == (4, 2, 2, 2, 4, 3)
    assert np.array_equal(synth.gaussian_spinors(L, 2)[1], synth.gaussian_spinor(L, 1001))
    b = synth.point_source_noise(L, 7, seed=5)
    assert abs(b[0, 0, 0, 0, 2, 1]) > 0.5


def test_haar_field_special_unitary():
    Om = synth.haar_su3_field((2, 2, 2, 2), seed=7)
    assert np.max(np.abs(Om @ np.conj(np.swapaxes(Om, -1, -2)) - np.eye(3))) < 1e-14
    assert np.max(np.abs(np.linalg.det(Om) - 1)) < 1e-13
