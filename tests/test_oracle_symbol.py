"""Pin for the circulant embedding of the Toeplitz block (Section 2.1)."""
import numpy as np
import scipy.linalg as sla

from oracle import allatonce as aa
from oracle.weights import gk_recurrence


def test_circulant_embedding_reproduces_toeplitz_product():
    for M, L in ((5, 16), (63, 128), (100, 256)):
        g = gk_recurrence(1.5, M)
        col = np.zeros(L)
        col[:M] = g
        col[L - M + 1:] = g[1:][::-1]
        Cmat = sla.circulant(col)
        assert np.allclose(Cmat, Cmat.T)
        ev = aa.circulant_symbol(g, M, L)
        x = np.random.default_rng(M).standard_normal(M)
        xp = np.concatenate([x, np.zeros(L - M)])
        # circulant product by its definition and by the eigen-decomposition
        assert np.allclose(Cmat @ xp, np.fft.ifft(ev * np.fft.fft(xp)).real, atol=1e-13)
        assert np.allclose((Cmat @ xp)[:M], sla.toeplitz(g) @ x, atol=1e-13)
