"""Pins of the network oracle: a layer with the Wilson weights is the Dirac
operator, gauge covariance, transport of plane waves, the adjoint (dot-product)
identity of the backward pass and central finite differences of the loss."""
import numpy as np
import pytest

from oracle import dirac, lattice
from oracle import network as net
from paper_1204_1306_amd import synth


def wilson_weights(kappa):
    W = np.zeros((9, 1, 1, 4, 4), np.complex128)
    W[0, 0, 0] = dirac.ONE4
    for mu in range(4):
        W[1 + 2 * mu, 0, 0] = -kappa * (dirac.ONE4 - dirac.GAMMA[mu])
        W[2 + 2 * mu, 0, 0] = -kappa * (dirac.ONE4 + dirac.GAMMA[mu])
    return W


def random_weights(rng, chans, scale=0.3):
    ws = []
    for cin, cout in zip(chans[:-1], chans[1:]):
        ws.append(scale * (rng.standard_normal((9, cout, cin, 4, 4)) + 1j * rng.standard_normal((9, cout, cin, 4, 4))))
    return ws


def test_layer_with_wilson_weights_is_the_dirac_operator():
    L = (4, 2, 4, 2)
    U = synth.gauge_field(L, 0.6, 3)
    psi = synth.gaussian_noise(L, 1, 4)[0]
    out = net.layer(U, wilson_weights(0.13), psi[None], L)[0]
    assert np.abs(out - dirac.apply_D(U, psi, 0.13, L)).max() < 1e-13


def test_transport_plane_wave_constant_links():
    L = (4, 4, 2, 2)
    rng = np.random.default_rng(5)
    th = rng.uniform(-1, 1, (4, 3))
    th[:, 2] = -th[:, 0] - th[:, 1]
    V = lattice.volume(L)
    U = np.zeros((V, 4, 3, 3), complex)
    for mu in range(4):
        U[:, mu] = np.diag(np.exp(1j * th[mu]))
    p = np.array([3 * np.pi / 4, np.pi / 2, np.pi, 0.0])
    x = lattice.coords(L)
    ph = np.exp(1j * (x @ p))
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    phi = ph[:, None, None] * u[None]
    for mu in range(4):
        f = net.transport(U, phi, 1 + 2 * mu, L)
        b = net.transport(U, phi, 2 + 2 * mu, L)
        assert np.abs(f - phi * np.exp(1j * (th[mu] + p[mu]))[None, None, :]).max() < 1e-13
        assert np.abs(b - phi * np.exp(-1j * (th[mu] + p[mu]))[None, None, :]).max() < 1e-13


def test_network_gauge_covariance():
    L = (4, 2, 2, 4)
    V = lattice.volume(L)
    rng = np.random.default_rng(7)
    U = synth.gauge_field(L, 0.6, 8)
    g = synth.gauge_transform(9, V)
    r = synth.gaussian_noise(L, 1, 10)[0]
    ws = random_weights(rng, [1, 3, 1])
    a, _ = net.forward(dirac.gauge_transform_links(U, g, L), ws, dirac.gauge_transform_spinor(r, g), L)
    b, _ = net.forward(U, ws, r, L)
    assert np.abs(a - dirac.gauge_transform_spinor(b, g)).max() < 1e-12


def test_pointwise_layer_is_spin_product():
    L = (2, 2, 2, 2)
    rng = np.random.default_rng(11)
    W = np.zeros((9, 1, 1, 4, 4), complex)
    W[0, 0, 0] = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    U = synth.gauge_field(L, 0.6, 12)
    psi = synth.gaussian_noise(L, 1, 13)[0]
    assert np.abs(net.layer(U, W, psi[None], L)[0] - np.matmul(W[0, 0, 0], psi)).max() < 1e-14


def test_backward_dot_product_identity():
    """<G, layer(Phi)> = <layer^dagger(G), Phi>: the input-gradient map is the adjoint."""
    L = (4, 2, 2, 2)
    rng = np.random.default_rng(14)
    U = synth.gauge_field(L, 0.6, 15)
    W = random_weights(rng, [2, 3])[0]
    phi = synth.gaussian_noise(L, 2, 16)
    G = synth.gaussian_noise(L, 3, 17)
    lhs = np.vdot(G, net.layer(U, W, phi, L))
    Gin = np.zeros_like(phi)
    for t in range(9):
        for ci in range(2):
            acc = sum(np.matmul(W[t, co, ci].conj().T, G[co]) for co in range(3))
            Gin[ci] += net.transport(U, acc, net.opposite(t), L)
    rhs = np.vdot(Gin, phi)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_gradient_central_differences():
    L = (2, 2, 2, 4)
    rng = np.random.default_rng(18)
    U = synth.gauge_field(L, 0.6, 19)
    ws = random_weights(rng, [1, 2, 2, 2, 1], scale=0.4)
    rs = list(synth.gaussian_noise(L, 2, 20))
    es = list(synth.gaussian_noise(L, 2, 21))
    _, grads = net.backward(U, ws, rs, es, L)
    h = 1e-6
    for l, idx in [(0, (3, 1, 0, 2, 1)), (1, (0, 1, 1, 0, 0)), (2, (6, 0, 1, 3, 2)), (3, (8, 0, 0, 1, 3))]:
        for part in (1.0, 1j):
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += h * part
            wm[l][idx] -= h * part
            fd = (net.loss(U, wp, rs, es, L) - net.loss(U, wm, rs, es, L)) / (2 * h)
            an = 2 * (grads[l][idx].real if part == 1.0 else grads[l][idx].imag)
            assert fd == pytest.approx(an, rel=1e-6, abs=1e-9)
