"""Pin of the device's interpolation tables against the paper's operators.

The GPU keeps, per box pair, the check potentials of B at A's check points
with B's corner phase divided out and rotated by E[k] = exp(-i pi rho k / q);
one level of step 3 then applies, per axis, T(s, t) = diag(sigma^s G(s, t, .))
R_t to the state of the child pair (A', B_s).  In the paper's terms
(Section 2.1) the same level is u^{AB} = sum_s E(A, B_s) M(A', B_s)^{-1}
u^{A'B_s}, with M from eq. (M1) and E from eq. (E1) written from the box
coordinates.  So, per axis,

    diag(sigma^s G(s, t, .)) R_t
        = Erot Phi(A, c_B) E(A, B_s) M(A', B_s)^{-1} Phi(A', c_{B_s})^{-1} Erot^{-1},

Phi(A, c) = diag(exp(-2 pi i x^A_l c / N)), Erot = diag(E[k]),
sigma = exp(2 pi i rho i_{A'}).  The right side is built here from the
coordinates in 40-digit mpmath (the paper's literal operators, no table
algebra), the left from the tables the plan built on the device (FP64),
at every p, for N a power of two (rho = 1) and not (rho < 1), at several
levels and box indices.
"""
import mpmath as mp
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0801_1524_amd as bf
    bf.lib()
    return bf


def literal_level_operator(N, L, p, ell, iAp, t, iB, s):
    """Per-axis operator of one level from the paper's M (eq. M1) and E
    (eq. E1), in the GPU's state convention (see the module docstring)."""
    mp.mp.dps = 40
    q = p - 1
    rho = mp.mpf(N) / mp.mpf(2) ** L
    wA, wAp = rho * 2 ** ell, rho * 2 ** (ell + 1)          # A at T_X level L - ell, A' its parent
    wB, wBs = rho * 2 ** (L - ell), rho * 2 ** (L - ell - 1)  # B at T_K level ell, B_s its child
    iA, iBs = 2 * iAp + t, 2 * iB + s
    cA, cAp, cB, cBs = iA * wA, iAp * wAp, iB * wB, iBs * wBs
    xA = [cA + l * wA / q for l in range(p)]
    xAp = [cAp + l * wAp / q for l in range(p)]
    kBs = [cBs + l * wBs / q for l in range(p)]
    e = lambda v: mp.expjpi(2 * v / N)
    E = mp.matrix(p, p)
    M = mp.matrix(p, p)
    for l in range(p):
        for m in range(p):
            E[l, m] = e(xA[l] * kBs[m])
            M[l, m] = e(xAp[l] * kBs[m])
    EMi = E * mp.inverse(M)
    T = np.zeros((p, p), dtype=np.complex128)
    for l in range(p):
        left = mp.expjpi(-rho * l / q) * e(-xA[l] * cB)
        for m in range(p):
            right = e(xAp[m] * cBs) / mp.expjpi(-rho * m / q)
            v = left * EMi[l, m] * right
            T[l, m] = complex(v)
    return T


@pytest.mark.parametrize("N", [256, 777])
@pytest.mark.parametrize("p", [3, 4, 5, 6, 7, 8, 9, 10, 11, 12])
def test_tables_equal_the_literal_operators(bf, N, p):
    x = np.array([[1.0, 2.0], [N - 3.0, N / 2.0]])
    with bf.Plan(2, N, p, x, x.copy(), "fp64") as plan:
        R, G, E = plan.tables()
        L = plan.info()["levels"]
    rho = N / 2.0 ** L
    rng = np.random.default_rng(N + p)
    worst = 0.0
    for ell in (0, 3, L - 2):
        for _ in range(2):
            iAp = int(rng.integers(0, 2 ** (L - ell - 1)))
            iB = int(rng.integers(0, 2 ** ell))
            # exp(2 pi i rho i_A'), rho i_A' = N i_A' / 2^L reduced exactly mod 1
            sigma = np.exp(2j * np.pi * ((N * iAp) % 2 ** L) / 2 ** L)
            for t in (0, 1):
                for s in (0, 1):
                    T = literal_level_operator(N, L, p, ell, iAp, t, iB, s)
                    Tg = (sigma ** s * G[s, t])[:, None] * R[t]
                    worst = max(worst, float(np.abs(Tg - T).max() / np.abs(T).max()))
    # FP64 tables (sine products, exact rational phases) against 40 digits
    assert worst <= 1e-13, worst
    # and the rotation itself
    q = p - 1
    assert np.abs(E - np.exp(-1j * np.pi * rho * np.arange(p) / q)).max() <= 1e-15
