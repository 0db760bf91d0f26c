"""Eigenvalue of largest real part of a linear operator by the Krylov-Schur method
(Stewart's restarted Arnoldi: expand the Krylov basis to m vectors, order the Schur form
of the projected matrix by real part, keep the leading `keep` Schur vectors, repeat).
Torch vectors, so one routine serves the oracle on the CPU and the library on the GPU.
Test infrastructure: it is pinned by the CPU tests against dense eigenvalues and the
free-field closed form.
"""
import numpy as np
import scipy.linalg


def krylov_schur_top_re(matvec, n, dev, m=48, keep=24, tol=1e-6, max_mv=12000, seed=0):
    """Eigenvalue of largest real part of the operator `matvec` (complex128 device
    vectors of length n) and its Ritz vector; returns (theta, v, matvecs)."""
    import torch

    V = torch.empty((m + 1, n), dtype=torch.complex128, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    v = torch.randn(n, dtype=torch.complex128, device=dev, generator=gen)
    V[0] = v / torch.linalg.vector_norm(v)
    Hm = np.zeros((m + 1, m), dtype=np.complex128)
    k, nmv = 0, 0
    while True:
        for j in range(k, m):
            w = matvec(V[j])
            nmv += 1
            h = torch.zeros(j + 1, dtype=torch.complex128, device=dev)
            for _ in range(2):  # classical Gram-Schmidt, twice
                c = (V[: j + 1] @ w.conj().resolve_conj()).conj().resolve_conj()
                w = w - c @ V[: j + 1]
                h = h + c
            beta = torch.linalg.vector_norm(w).item()
            Hm[: j + 1, j] = h.cpu().numpy()
            Hm[j + 1, j] = beta
            V[j + 1] = w / beta
        theta, Y = np.linalg.eig(Hm[:m, :m])
        top = int(np.argmax(theta.real))
        y = Y[:, top] / np.linalg.norm(Y[:, top])
        res = abs(Hm[m, :m] @ y)
        if res <= tol * abs(theta[top]) or nmv >= max_mv:
            yt = torch.from_numpy(y).to(dev)
            return theta[top], yt @ V[:m], nmv
        thr = np.sort(theta.real)[::-1][keep - 1]
        T, Z, p = scipy.linalg.schur(Hm[:m, :m], output="complex", sort=lambda x: x.real >= thr)
        p = min(max(p, 1), m - 1)
        Zp = torch.from_numpy(np.ascontiguousarray(Z[:, :p].T)).to(dev)
        V[:p] = Zp @ V[:m]
        V[p] = V[m]
        b = Hm[m, :m] @ Z[:, :p]
        Hm[:] = 0
        Hm[:p, :p] = T[:p, :p]
        Hm[p, :p] = b
        k = p
