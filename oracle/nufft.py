"""Measurement operator and data-fidelity dual update (oracle).

TEST INFRASTRUCTURE ONLY.

Per channel l (Sec. 2.1, eq. model): Phi_l = G_l F Z, with
  Z  zero-padding and scaling of the ny x nx image into a K1 x K2 grid
     (K = 2 N per axis), the image centred on the grid origin: pixel n goes
     to grid index (n - N/2) mod K, multiplied by 1 / Psi^(m / K) per axis
     (m = n - N/2), Psi^ the continuous Fourier transform of the interpolation
     kernel;
  F  the unnormalised 2D DFT of the grid, X^[k] = sum_g Z[g] exp(-2 pi i k.g / K);
  G  de-gridding: visibility j at the uv-point omega_j (radians per pixel, in
     [-pi, pi)^2) sits at grid coordinate t = omega K / (2 pi); it is
     sum over the J x J nearest grid points k of psi(t_y - k_y) psi(t_x - k_x)
     X^[k mod K], with the Kaiser-Bessel kernel of width J = 7
     psi(d) = I0(beta sqrt(1 - (2 d / J)^2)) for |d| <= J / 2 (Sec. 2.1 and
     Sec. 4.1: 7 x 7 Kaiser-Bessel kernels), beta from the oversampling
     factor (Beatty, Nishimura and Pauly 2005):
     beta = pi sqrt((J / alpha)^2 (alpha - 1/2)^2 - 0.8), alpha = 2.
So Phi x approximates the centred DFT y(omega) = sum_n x[n] exp(-i omega.(n - N/2)).
The adjoint of a real image's operator is Re(Z^T F^H G^H v).

The data-fidelity dual update of Alg. 2 (one data block per channel):
  z      = U^-1 v + Phi x_check     (2 x^(p+1) - x^(p) in the Fourier domain is
                                      the transform of the extrapolated iterate)
  v+     = U (z - prox^U_{ball}(z)), prox^U the projection onto the l2 ball
           B(y, eps) in the metric of the diagonal U (eq. prox_definition),
           approximated by forward-backward sub-iterations that each take one
           Euclidean projection onto the ball (Sec. 3.2)
  a     += eta Re Phi^dagger v+     (the data part of the aggregation)
  r      = ||y - Phi x||             (the residual of the iterate)
U holds the inverse sampling density: 1 / (number of uv-points in the point's
cell of the oversampled grid) (Sec. 3.2, preconditioning).
"""
import numpy as np

KB_WIDTH = 7
OVERSAMPLE = 2


def kb_beta(J=KB_WIDTH, alpha=OVERSAMPLE):
    return np.pi * np.sqrt((J / alpha) ** 2 * (alpha - 0.5) ** 2 - 0.8)


def kb_kernel(d, J=KB_WIDTH, beta=None):
    """psi(d), zero outside |d| <= J / 2."""
    beta = kb_beta(J) if beta is None else beta
    d = np.asarray(d, dtype=np.float64)
    a = 1.0 - (2.0 * d / J) ** 2
    return np.where(a >= 0.0, np.i0(beta * np.sqrt(np.maximum(a, 0.0))), 0.0)


def kb_fourier(xi, J=KB_WIDTH, beta=None):
    """Psi^(xi) = integral of psi(d) exp(2 pi i d xi) dd (psi is even): the
    closed form J sinh(sqrt(beta^2 - (pi J xi)^2)) / sqrt(beta^2 - (pi J xi)^2)
    (sin for the imaginary root)."""
    beta = kb_beta(J) if beta is None else beta
    z = np.sqrt(beta ** 2 - (np.pi * J * np.asarray(xi, dtype=np.float64)) ** 2 + 0j)
    return np.real(J * np.sinh(z) / z)


def centred(N):
    """Pixel offsets n - N/2 of an axis of N pixels."""
    return np.arange(N) - N // 2


def interp_1d(t, K, J=KB_WIDTH):
    """First grid index and the J weights of each coordinate t (grid units)."""
    k0 = np.ceil(t - J / 2.0).astype(np.int64)
    ks = k0[:, None] + np.arange(J)[None, :]
    return k0, kb_kernel(t[:, None] - ks, J)


class Nufft:
    """Phi = G F Z for one ny x nx image and M uv-points omega (M, 2) =
    (omega_y, omega_x) in radians per pixel."""

    def __init__(self, ny, nx, omega, J=KB_WIDTH, alpha=OVERSAMPLE):
        self.ny, self.nx, self.J = ny, nx, J
        self.K1, self.K2 = alpha * ny, alpha * nx
        self.omega = np.asarray(omega, dtype=np.float64)
        self.s1 = 1.0 / kb_fourier(centred(ny) / self.K1, J)
        self.s2 = 1.0 / kb_fourier(centred(nx) / self.K2, J)
        t1 = self.omega[:, 0] * self.K1 / (2 * np.pi)
        t2 = self.omega[:, 1] * self.K2 / (2 * np.pi)
        self.k1, self.w1 = interp_1d(t1, self.K1, J)
        self.k2, self.w2 = interp_1d(t2, self.K2, J)

    def zf(self, x):
        """F Z x: the oversampled spectrum (K1, K2) of the image x (ny, nx)."""
        g = np.zeros((self.K1, self.K2), dtype=np.complex128)
        g[np.ix_(centred(self.ny) % self.K1, centred(self.nx) % self.K2)] = \
            np.asarray(x, dtype=np.float64) * self.s1[:, None] * self.s2[None, :]
        return np.fft.fft2(g)

    def degrid(self, X):
        """G X: the M visibilities from the spectrum."""
        J = self.J
        r1 = (self.k1[:, None, None] + np.arange(J)[None, :, None]) % self.K1
        r2 = (self.k2[:, None, None] + np.arange(J)[None, None, :]) % self.K2
        w = self.w1[:, :, None] * self.w2[:, None, :]
        return np.sum(w * X[r1, r2], axis=(1, 2))

    def forward(self, x):
        return self.degrid(self.zf(x))

    def adjoint(self, v):
        """Re(Z^T F^H G^H v): the real image (ny, nx)."""
        J = self.J
        g = np.zeros((self.K1, self.K2), dtype=np.complex128)
        r1 = (self.k1[:, None, None] + np.arange(J)[None, :, None]) % self.K1
        r2 = (self.k2[:, None, None] + np.arange(J)[None, None, :]) % self.K2
        w = self.w1[:, :, None] * self.w2[:, None, :]
        np.add.at(g, (r1, r2), w * np.asarray(v, dtype=np.complex128)[:, None, None])
        # F^H = conj(F) (unnormalised inverse DFT times K1 K2)
        G = np.fft.ifft2(g) * (self.K1 * self.K2)
        img = G[np.ix_(centred(self.ny) % self.K1, centred(self.nx) % self.K2)]
        return np.real(img) * self.s1[:, None] * self.s2[None, :]


def nudft(x, omega):
    """The centred DFT sum_n x[n] exp(-i omega.(n - N/2)), brute force."""
    ny, nx = x.shape
    my, mx = centred(ny), centred(nx)
    ey = np.exp(-1j * np.outer(omega[:, 0], my))
    ex = np.exp(-1j * np.outer(omega[:, 1], mx))
    return np.einsum("jy,yx,jx->j", ey, np.asarray(x, dtype=np.float64), ex)


def inverse_density(omega, K1, K2):
    """U_j = 1 / (number of uv-points in point j's cell of the K1 x K2 grid,
    the cell of the nearest grid point)."""
    c1 = np.rint(omega[:, 0] * K1 / (2 * np.pi)).astype(np.int64) % K1
    c2 = np.rint(omega[:, 1] * K2 / (2 * np.pi)).astype(np.int64) % K2
    cell = c1 * K2 + c2
    _, inv, counts = np.unique(cell, return_inverse=True, return_counts=True)
    return 1.0 / counts[inv]


def project_ball(z, y, eps):
    """Euclidean projection onto B(y, eps)."""
    d = z - y
    n = np.linalg.norm(d)
    return z.copy() if n <= eps else y + d * (eps / n)


def project_ball_metric(z, y, eps, U, tol=1e-15):
    """Projection onto B(y, eps) in the metric of the diagonal U > 0, exactly:
    p = (U z + lam y) / (U + lam), lam >= 0 with ||p - y|| = eps (the KKT
    conditions), found by bisection (||p(lam) - y|| decreases in lam)."""
    if np.linalg.norm(z - y) <= eps:
        return z.copy()
    U = np.asarray(U, dtype=np.float64)

    def dist(lam):
        return np.linalg.norm(U * (z - y) / (U + lam))

    lo, hi = 0.0, 1.0
    while dist(hi) > eps:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if dist(mid) > eps:
            lo = mid
        else:
            hi = mid
        if hi - lo <= tol * hi:
            break
    lam = hi
    return (U * z + lam * y) / (U + lam)


def project_ball_metric_fb(z, y, eps, U, n_sub):
    """The same projection by forward-backward sub-iterations (Sec. 3.2): the
    objective 1/2 (p - z)^H U (p - z) over the ball, step gamma = 1 / max U;
    each sub-iteration p <- P_B(p - gamma U (p - z)) takes one Euclidean
    projection.  Starts from P_B(z); n_sub = 0 returns P_B(z)."""
    U = np.asarray(U, dtype=np.float64)
    if U.size == 0:                      # an empty data block: nothing to project
        return np.asarray(z).copy()
    gamma = 1.0 / np.max(U)
    p = project_ball(z, y, eps)
    for _ in range(n_sub):
        p = project_ball(p - gamma * U * (p - z), y, eps)
    return p


def data_dual_update(x, xcheck, v, y, U, eps, eta, n_sub, ops):
    """Alg. 2 data-fidelity lines for every channel l (one block each).

    x, xcheck: (ny, nx, L) real; v, y: lists of (M_l,) complex; U: list of
    (M_l,) real; eps, eta: (L,); ops: list of Nufft per channel.
    Returns (v_new list, grad (ny, nx, L) = eta_l Re Phi_l^dagger v_new_l,
    residual (L,) = ||y_l - Phi_l x_l||).
    """
    L = x.shape[2]
    v_new, res = [], np.zeros(L)
    grad = np.zeros(x.shape)
    for l in range(L):
        op = ops[l]
        z = np.asarray(v[l], dtype=np.complex128) / U[l] + op.forward(xcheck[..., l])
        p = project_ball_metric_fb(z, np.asarray(y[l], dtype=np.complex128), eps[l], U[l], n_sub)
        vn = U[l] * (z - p)
        v_new.append(vn)
        grad[..., l] = eta[l] * op.adjoint(vn)
        res[l] = np.linalg.norm(np.asarray(y[l], dtype=np.complex128) - op.forward(x[..., l]))
    return v_new, grad, res
