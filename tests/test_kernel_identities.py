"""Identities the GPU kernels are built on, checked in plain numpy on the CPU (no GPU, no
oracle): the half-length DST-I of the 1D tau solve, the chirp-z DST-I of any length, the
factored Arnoldi basis of the two-sweep CGS2, Durbin's recursion without conjugation with the
Gohberg-Semencul inverse of a complex symmetric Toeplitz matrix (by transforms, and by the
direct sums the application uses for a row it does not transform), the one-pass-per-step
organisation of that recursion in the setup kernel, and the Gram-Schmidt/Givens form of GMRES
in the 2D inner solver.  The GPU parity tests check the kernels themselves against the
oracle."""
import numpy as np
import pytest


def _sine_sums(x):
    """S_m = sum_j x_j sin(pi j m / N), m = 1..N-1, by definition (N = len(x) + 1)."""
    n = len(x)
    N = n + 1
    j = np.arange(1, N)
    return np.sin(np.pi * np.outer(j, j) / N) @ x


def _sine_sums_half(x):
    """The same sums through one complex FFT of length N: c_j = sin(pi j / N)(x_j + x_{N-j}) +
    (x_j - x_{N-j}) / 2, F_k = sum_j c_j exp(+2 pi i j k / N); S_{2k} = -i (F_k - F_{N-k}) / 2,
    S_{2k+1} = sum_{q <= k} (F_q + F_{N-q}) / 2 - F_0 / 2."""
    n = len(x)
    N = n + 1
    xx = np.zeros(N + 1, dtype=complex)
    xx[1:N] = x
    j = np.arange(N)
    c = np.sin(np.pi * j / N) * (xx[j] + xx[N - j]) + 0.5 * (xx[j] - xx[N - j])
    F = np.fft.ifft(c) * N
    k = np.arange(N // 2)
    Fm = F[(N - k) % N]
    O = (F[k] + Fm) / 2
    E = -1j * (F[k] - Fm) / 2
    S = np.zeros(N, dtype=complex)
    S[2 * k[1:]] = E[1:]
    S[2 * k + 1] = np.cumsum(O) - F[0] / 2
    return S[1:]


@pytest.mark.parametrize("n", [3, 7, 15, 255, 1023])
def test_half_length_dst(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = _sine_sums(x)
    assert np.abs(_sine_sums_half(x) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_factored_cgs2_basis():
    # two sweeps over the stored vectors U (after the first projection), V = U R^{-1} with the
    # inverse factor kept: the Hessenberg matrix is classic CGS2's and A Z = V H holds
    rng = np.random.default_rng(7)
    n, m = 300, 24
    A = np.eye(n) + 0.4 * rng.standard_normal((n, n)) / np.sqrt(n)
    P = np.diag(1.0 + rng.random(n))  # a fixed "preconditioner" direction map
    r = rng.standard_normal(n)
    beta = np.linalg.norm(r)
    # classic CGS2 on a normalised basis
    V = np.zeros((n, m + 1))
    V[:, 0] = r / beta
    H = np.zeros((m + 1, m))
    for j in range(m):
        w = A @ (P @ V[:, j])
        h1 = V[:, : j + 1].T @ w
        w1 = w - V[:, : j + 1] @ h1
        h2 = V[:, : j + 1].T @ w1
        w2 = w1 - V[:, : j + 1] @ h2
        H[: j + 1, j] = h1 + h2
        H[j + 1, j] = np.linalg.norm(w2)
        V[:, j + 1] = w2 / H[j + 1, j]
    # factored: U, Q = R^{-1}, unit-scaled inputs u_j / |u_j|
    U = np.zeros((n, m + 1))
    U[:, 0] = r
    Q = np.zeros((m + 1, m + 1))
    Q[0, 0] = 1 / beta
    vs = np.zeros(m + 1)
    vs[0] = 1 / beta
    H2 = np.zeros((m + 1, m))
    Z = np.zeros((n, m))
    for j in range(m):
        k = j + 1
        Z[:, j] = P @ (U[:, j] * vs[j])
        w = A @ Z[:, j]
        h1 = Q[:k, :k].T @ (U[:, :k].T @ w)
        c1 = Q[:k, :k] @ h1
        w1 = w - U[:, :k] @ c1
        s = w1 @ w1
        h2 = Q[:k, :k].T @ (U[:, :k].T @ w1)
        nn = np.sqrt(s - h2 @ h2)
        Q[:k, k] = -(Q[:k, :k] @ h2) / nn
        Q[k, k] = 1 / nn
        U[:, k] = w1
        vs[k] = 1 / np.sqrt(s)
        H2[:k, j] = h1 + h2
        H2[k, j] = nn
    Vimp = U @ Q
    assert np.abs(Vimp.T @ Vimp - np.eye(m + 1)).max() < 1e-13
    assert np.abs(A @ Z - Vimp @ H2).max() < 1e-13 * np.abs(A @ Z).max()
    # the directions differ from classic CGS2's only by the unapplied second projection of
    # u_j, so the Hessenberg matrices agree to rounding level
    assert np.abs(H2 - H).max() < 1e-12 * np.abs(H).max()


def _dst_chirp_z(x):
    """The sine sums S_k = sum_j x_j sin(pi j k/(n+1)), k = 1..n, as the chirp-z DST-I kernel
    forms them: S = (P - Q)/(2i) with P_k = c_k sum_j (x_j c_j) conj(c_{k-j}) and
    Q_k = conj(c_k) sum_j (x_j conj(c_j)) c_{k-j}, c_m = exp(i pi (m^2 mod 4(n+1)) / (2(n+1))),
    each a cyclic convolution of length LB >= 2n - 1 with the kernel transform Khat (that of
    conj(c_m)) for P and conj(Khat[(LB - k) mod LB]) for Q."""
    n = len(x)
    LB = 8
    while LB < 2 * n - 1:
        LB *= 2
    m = np.arange(n + 1)
    c = np.exp(1j * np.pi * ((m * m) % (4 * (n + 1))) / (2.0 * (n + 1)))
    b = np.zeros(LB, dtype=complex)
    b[:n] = np.conj(c[:n])
    b[LB - np.arange(1, n)] = np.conj(c[1:n])
    Khat = np.fft.fft(b) / LB
    a = np.zeros(LB, dtype=complex)
    a[1:n + 1] = x * c[1:]
    P = np.fft.ifft(np.fft.fft(a) * Khat) * LB
    a2 = np.zeros(LB, dtype=complex)
    a2[1:n + 1] = x * np.conj(c[1:])
    K2 = np.conj(Khat[(LB - np.arange(LB)) % LB])
    Q = np.fft.ifft(np.fft.fft(a2) * K2) * LB
    k = np.arange(1, n + 1)
    return ((P[k] * c[k]) - (Q[k] * np.conj(c[k]))) / 2j


@pytest.mark.parametrize("n", [1, 2, 5, 59, 60, 100, 255, 1000, 2730, 4096])
def test_chirp_z_dst(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = _sine_sums(x)
    got = _dst_chirp_z(x)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref))) * np.log2(4 * n + 8)


def _durbin_first_column(t):
    """First column of T^-1 for the complex symmetric Toeplitz T of first column t, by Durbin's
    recursion on T / t_0 (no conjugation), as the setup kernel runs it."""
    n = len(t)
    if n == 1:
        return np.array([1.0 / t[0]])
    r = t[1:] / t[0]
    y = np.zeros(n - 1, dtype=complex)
    a = -r[0]
    y[0] = a
    beta = 1.0 + 0j
    for k in range(1, n - 1):
        beta = (1 - a * a) * beta
        a = -(r[k] + np.dot(r[k - 1::-1][:k], y[:k])) / beta
        yk = y[:k].copy()
        y[:k] = yk + a * yk[::-1]
        y[k] = a
    gamma = 1.0 / (1.0 + np.dot(r, y))
    return gamma / t[0] * np.concatenate([[1.0], y])


def _gohberg_semencul_apply(x, b, L):
    """T^-1 b = (L(x) L(x)^T b - L(u) L(u)^T b) / x_0, u = (0, x_{n-1}, .., x_1), with the four
    triangular Toeplitz products as truncated cyclic convolutions of length L, the transform of
    u taken from that of x (DFT(u)_k = w^{nk} (X_{-k} - x_0)), and L(v)^T = J L(v) J."""
    n = len(x)
    X = np.fft.fft(np.concatenate([x, np.zeros(L - n)])) / L
    k = np.arange(L)
    U = np.exp(-2j * np.pi * ((n * k) % L) / L) * (X[(L - k) % L] - x[0] / L)

    def conv(v, S):
        V = np.fft.fft(np.concatenate([v, np.zeros(L - len(v))]))
        return (np.fft.ifft(V * S) * L)[:n]

    p = conv(b[::-1], X)[::-1]
    q = conv(b[::-1], U)[::-1]
    return (conv(p, X) - conv(q, U)) / x[0]


@pytest.mark.parametrize("n", [1, 2, 7, 63, 100, 511])
def test_durbin_gohberg_semencul(n):
    # a symmetric positive definite Toeplitz T (first column from a positive spectral density)
    # plus a complex shift with positive real part: B = lam I + T, complex symmetric
    rng = np.random.default_rng(n)
    th = rng.uniform(0, np.pi, 8)
    wts = rng.uniform(0.1, 1.0, 8)
    t = np.array([np.sum(wts * np.cos(k * th)) for k in range(n)], dtype=complex)
    t[0] += 0.05 + 0.3j
    B = np.array([[t[abs(i - j)] for j in range(n)] for i in range(n)])
    x = _durbin_first_column(t)
    assert np.allclose(B @ x, np.eye(n)[:, 0], atol=1e-12)
    L = 16
    while L < 2 * n - 1:
        L *= 2
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    z = _gohberg_semencul_apply(x, b, L)
    ref = np.linalg.solve(B, b)
    assert np.max(np.abs(z - ref)) < 1e-10 * np.max(np.abs(ref))


def _gohberg_semencul_direct(x, b, lanes=64):
    """The same inverse by direct sums, as the application kernels form the row they do not
    transform: p_m = sum_{l >= m} x_{l-m} b_l, q_m = sum_{l > m} x_{n-(l-m)} b_l, then
    z_i = (sum_{j <= i} x_{i-j} p_j - sum_{j < i} x_{n-(i-j)} q_j) / x_0; each sum split over
    `lanes` lanes (lane c takes terms c, c + lanes, ...) in four interleaved partial sums per
    lane, the lanes' totals then added."""
    n = len(x)

    def lane_sum(cnt, term):
        tot = 0
        for c in range(lanes):
            s = [0, 0, 0, 0]
            t = c
            while t + 3 * lanes < cnt:
                for r in range(4):
                    s[r] += term(t + r * lanes)
                t += 4 * lanes
            while t < cnt:
                s[0] += term(t)
                t += lanes
            tot += (s[0] + s[1]) + (s[2] + s[3])
        return tot

    p = np.array([lane_sum(n - m, lambda d: x[d] * b[m + d]) for m in range(n)])
    q = np.array([lane_sum(n - m - 1, lambda e: x[n - 1 - e] * b[m + 1 + e]) for m in range(n)])
    z = [lane_sum(i + 1, lambda j: x[i - j] * p[j]) - lane_sum(i, lambda j: x[n - (i - j)] * q[j])
         for i in range(n)]
    return np.array(z) / x[0]


@pytest.mark.parametrize("n,lanes", [(1, 64), (2, 64), (9, 4), (40, 4), (300, 8), (300, 64)])
def test_gohberg_semencul_direct_sums(n, lanes):
    rng = np.random.default_rng(200 + n)
    th = rng.uniform(0, np.pi, 8)
    wts = rng.uniform(0.1, 1.0, 8)
    t = np.array([np.sum(wts * np.cos(k * th)) for k in range(n)], dtype=complex)
    t[0] += 0.05 + 0.3j
    B = np.array([[t[abs(i - j)] for j in range(n)] for i in range(n)])
    x = np.linalg.solve(B, np.eye(n)[:, 0])
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.linalg.solve(B, b)
    z = _gohberg_semencul_direct(x, b, lanes)
    assert np.max(np.abs(z - ref)) < 1e-10 * np.max(np.abs(ref))


def _durbin_one_pass(t, NT=4, S=8):
    """Durbin's recursion as the setup kernel organises it (one pass and one block sum per
    step): the thread of pair (i, k+1-i), i = 1 + t + NT q, updates both entries and adds their
    terms of the next step's sum g_{k+2-i} y_i + g_{i+1} y_j (y_i once when i = j); y_i stays
    in the thread's register from the step it joins the lower half (2i <= k+1); the partner
    weights g_{k+2-i} are loaded a step ahead, reading zero outside [0, n) for the slots not yet
    active."""
    n = len(t)
    if n == 1:
        return np.array([1.0 / t[0]])
    g = t / t[0]  # r_k = g_k for k >= 1 (g_0 = 1)
    G = lambda m: g[m] if 0 <= m < n else 0.0
    lds = np.full(n - 1, np.nan, dtype=complex)
    reg = np.zeros((NT, S), dtype=complex)
    idx = np.array([[1 + th + NT * q for q in range(S)] for th in range(NT)])
    gi = np.vectorize(lambda i: G(i + 1), otypes=[complex])(idx)
    gj = np.vectorize(lambda i: G(3 - i), otypes=[complex])(idx)
    a = -g[1]
    lds[0] = a
    beta = 1.0 + 0j
    dot = g[1] * a
    for k in range(1, n - 1):
        beta = (1 - a * a) * beta
        a = -(dot + g[k + 1]) / beta
        old = lds.copy()
        acc = 0
        for th in range(NT):
            for q in range(S):
                i = idx[th, q]
                if 2 * i > k + 1:
                    continue
                yj = old[k - i]
                first = 2 * i == k + 1
                yi = yj if first else reg[th, q]
                ni, nj = yi + a * yj, yj + a * yi
                reg[th, q] = ni
                if not first:
                    lds[k - i] = nj
                acc += gj[th, q] * ni + (0 if first else gi[th, q]) * nj
        lds[k] = a
        # partner weights of step k + 1: g_{k+3-i}
        gj = np.vectorize(lambda i: G(k + 3 - i), otypes=[complex])(idx)
        dot = acc + g[1] * a
    for th in range(NT):
        for q in range(S):
            i = idx[th, q]
            if 2 * i <= n - 1:
                lds[i - 1] = reg[th, q]
    gamma = 1.0 / (1.0 + np.dot(g[1:], lds))
    return gamma / t[0] * np.concatenate([[1.0], lds])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 17, 40, 64])
def test_durbin_one_pass_matches_plain_recursion(n):
    rng = np.random.default_rng(100 + n)
    th = rng.uniform(0, np.pi, 8)
    wts = rng.uniform(0.1, 1.0, 8)
    t = np.array([np.sum(wts * np.cos(k * th)) for k in range(n)], dtype=complex)
    t[0] += 0.05 + 0.3j
    ref = _durbin_first_column(t)
    got = _durbin_one_pass(t)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def _gmres_cgs2_givens(C, w, k):
    """k GMRES steps from zero for C x = w as the 2D inner-solver kernels do them: classical
    Gram-Schmidt twice with Hermitian products, h_{j+1,j} = sqrt(||w||^2 - ||h2||^2) after the
    second projection, complex Givens rotations with a real cosine
    (c = |a| / rho, s = (a / |a|) h / rho), y = R^-1 g."""
    n = len(w)
    beta = np.linalg.norm(w)
    V = [w / beta]
    R = np.zeros((k + 1, k), dtype=complex)
    cs = np.zeros(k)
    sn = np.zeros(k, dtype=complex)
    g = np.zeros(k + 1, dtype=complex)
    g[0] = beta
    for j in range(k):
        x = C @ V[j]
        Vm = np.stack(V, axis=1)
        h1 = Vm.conj().T @ x
        x = x - Vm @ h1
        h2 = Vm.conj().T @ x
        s2 = np.vdot(x, x).real
        x = x - Vm @ h2
        hn = np.sqrt(max(s2 - np.vdot(h2, h2).real, 0.0))
        h = np.zeros(k + 1, dtype=complex)
        h[: j + 1] = h1 + h2
        h[j + 1] = hn
        for i in range(j):
            a, b = h[i], h[i + 1]
            h[i] = cs[i] * a + sn[i] * b
            h[i + 1] = cs[i] * b - np.conj(sn[i]) * a
        a = h[j]
        rho = np.hypot(abs(a), hn)
        ph = a / abs(a) if abs(a) > 0 else 1.0
        cs[j], sn[j] = abs(a) / rho, ph * hn / rho
        R[: j + 1, j] = h[: j + 1]
        R[j, j] = ph * rho
        gj = g[j]
        g[j] = cs[j] * gj
        g[j + 1] = -np.conj(sn[j]) * gj
        V.append(x / hn)
    y = np.linalg.solve(np.triu(R[:k, :k]), g[:k])
    return np.stack(V[:k], axis=1) @ y, abs(g[k])


@pytest.mark.parametrize("k", [1, 2, 5, 12])
def test_inner_gmres_givens_matches_least_squares(k):
    # the residual estimate |g_k| and x = V y equal the minimiser of ||w - C x|| over the
    # Krylov space (brute force on an orthonormalised power basis)
    rng = np.random.default_rng(k)
    n = 40
    C = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    w = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, est = _gmres_cgs2_givens(C, w, k)
    K = np.stack([np.linalg.matrix_power(C, i) @ w for i in range(k)], axis=1)
    Qk, _ = np.linalg.qr(K)
    c = np.linalg.lstsq(C @ Qk, w, rcond=None)[0]
    ref = Qk @ c
    assert np.max(np.abs(x - ref)) < 1e-10 * np.max(np.abs(ref))
    assert abs(est - np.linalg.norm(w - C @ x)) < 1e-10 * np.linalg.norm(w)
