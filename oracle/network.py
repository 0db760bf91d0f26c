"""FP64 oracle of the gauge-covariant linear network used as a preconditioner.

Not from the paper: the learned preconditioner wraps the paper's solves. A layer
maps C_in spinor channels to C_out channels,

    Psi_c(x) = sum_{t=0..8} sum_{c'} W[t, c, c'] (T_t Phi_{c'})(x),

with the parallel transports T_0 = 1, T_{1+2mu} Phi(x) = U(x,mu) Phi(x+mu) and
T_{2+2mu} Phi(x) = U(x-mu,mu)^dagger Phi(x-mu) (with the fermion boundary sign
across the time boundary, as in the Dirac operator), and W[t, c, c'] a complex
4x4 matrix acting on spin (identity on colour). Every layer commutes with gauge
transformations. The network is a chain of such layers, linear in its input.

Gradients use the Wirtinger convention for the real loss
L = sum_b |N(r_b) - e_b|^2 / |e_b|^2: G = dL/dconj(Psi), and for a layer
dL/dconj(W[t,c,c'])[s,s'] = sum_{x,a} G_c(x)[s,a] conj((T_t Phi_{c'})(x)[s',a]),
dL/dconj(Phi_{c'}) = sum_t sum_c T_t^dagger (W[t,c,c']^dagger G_c),
with T_{1+2mu}^dagger = T_{2+2mu}.
"""
from __future__ import annotations

import numpy as np


def _grid(L, a, tail):
    return a.reshape(tuple(L) + tail)


def transport(U: np.ndarray, phi: np.ndarray, t: int, L, antiperiodic: bool = True) -> np.ndarray:
    """T_t phi for one spinor field phi[V, 4, 3]."""
    if t == 0:
        return phi.copy()
    mu = (t - 1) // 2
    fwd = (t - 1) % 2 == 0
    P = _grid(L, phi, (4, 3))
    Umu = _grid(L, U, (4, 3, 3))[..., mu, :, :]
    if fwd:
        nb = np.roll(P, -1, axis=mu)
        if antiperiodic and mu == 0:
            nb[-1] = -nb[-1]
        out = np.matmul(nb, np.swapaxes(Umu, -1, -2))           # U(x,mu) phi(x+mu)
    else:
        nb = np.roll(P, 1, axis=mu)
        if antiperiodic and mu == 0:
            nb[0] = -nb[0]
        out = np.matmul(nb, np.roll(Umu, 1, axis=mu).conj())    # U(x-mu,mu)^dagger phi(x-mu)
    return out.reshape(phi.shape)


def opposite(t: int) -> int:
    return 0 if t == 0 else (t + 1 if t % 2 == 1 else t - 1)


def layer(U, W: np.ndarray, phi: np.ndarray, L, antiperiodic=True) -> np.ndarray:
    """One layer: W[9, C_out, C_in, 4, 4], phi[C_in, V, 4, 3] -> [C_out, V, 4, 3]."""
    cout, cin = W.shape[1], W.shape[2]
    out = np.zeros((cout,) + phi.shape[1:], np.complex128)
    for t in range(9):
        for ci in range(cin):
            tp = transport(U, phi[ci], t, L, antiperiodic)
            for co in range(cout):
                out[co] += np.matmul(W[t, co, ci], tp)
    return out


def forward(U, weights, r: np.ndarray, L, antiperiodic=True):
    """Network output for input r[V, 4, 3]; returns (output[V,4,3], activations)."""
    acts = [r[None]]
    for W in weights:
        acts.append(layer(U, W, acts[-1], L, antiperiodic))
    return acts[-1][0], acts


def loss(U, weights, rs, es, L, antiperiodic=True) -> float:
    return float(sum(np.sum(np.abs(forward(U, weights, r, L, antiperiodic)[0] - e) ** 2) / np.sum(np.abs(e) ** 2)
                     for r, e in zip(rs, es)))


def backward(U, weights, rs, es, L, antiperiodic=True):
    """Loss and dL/dconj(W) for every layer (analytic, Wirtinger convention)."""
    grads = [np.zeros_like(W) for W in weights]
    total = 0.0
    for r, e in zip(rs, es):
        out, acts = forward(U, weights, r, L, antiperiodic)
        en = np.sum(np.abs(e) ** 2)
        total += np.sum(np.abs(out - e) ** 2) / en
        G = ((out - e) / en)[None]
        for l in range(len(weights) - 1, -1, -1):
            W = weights[l]
            phi = acts[l]
            cout, cin = W.shape[1], W.shape[2]
            for t in range(9):
                for ci in range(cin):
                    tp = transport(U, phi[ci], t, L, antiperiodic)
                    for co in range(cout):
                        # sum over sites and colour of G[s,a] conj(tp[s',a])
                        grads[l][t, co, ci] += np.einsum("xsa,xta->st", G[co], tp.conj())
            if l > 0:
                Gin = np.zeros((cin,) + G.shape[1:], np.complex128)
                for t in range(9):
                    for ci in range(cin):
                        acc = np.zeros(G.shape[1:], np.complex128)
                        for co in range(cout):
                            acc += np.matmul(W[t, co, ci].conj().T, G[co])
                        Gin[ci] += transport(U, acc, opposite(t), L, antiperiodic)
                G = Gin
    return float(total), grads
