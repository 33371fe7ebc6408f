"""FP64 CPU oracle for cross-correlation particle tracking.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain statement of what
the tracker computes, used to check the GPU library.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it; the
product path never calls it and shares no code with it.

Every quantity is computed in float64 with numpy.  Steps follow the paper
(arXiv 2310.08770, "Cross-correlation image analysis for real-time single
particle tracking"):

  O1 weights       Sec. II, Eq. (2)-(7) and the substitution rule of Sec. III
  O2 cross-power   Eq. (4) / Eq. (7): X = F[A] * conj(F[B])
  O3 correlation   inverse transform of X
  O4 integer peak  Sec. III, first paragraph: argmax of the correlation
  O5 band-limited correlation C(s) (trigonometric interpolant of the
                   correlation; the paper's upsampled DFT samples it)
  O6 upsampled grid Sec. III, first paragraph: 1.5-px square, 1.5u points
                   per axis, centred on the integer peak; its argmax is the
                   paper's sub-pixel estimate d_grid
  O7 Newton        refinement of d_grid to the maximiser of C(s) (the paper
                   stops at the grid; see the readings below)
  O8 adjoint       gradient of (d_hat, C(d_hat)) with respect to frame and
                   reference by the implicit function theorem
  O9 Fisher / CRB  Cramer-Rao bound of the displacement under Poisson noise
                   (the shot-noise limit of Sec. IV)
  O10 offline reference  Sec. III.A, Eq. (8): the reference as the mean of
                   all frames shifted back by their displacements, in Fourier
                   space, iterated pass by pass from F[E_0] = F[I_0]
  O11 real-time reference  Sec. III.B, Eq. (9): low-pass update of the
                   reference spectrum by each tracked frame shifted back
  O12 drift correction  Sec. III.B, Eq. (10)-(12): low-pass offset of the
                   displacement stream, optionally rate-limited to alpha/u

Readings where the paper is silent or loose (each is also listed in the
design notes of the repository):

* Sign (Eq. 4).  The inverse transform of F[I] conj(F[E]) at lag s equals
  sum_r I(r+s) E(r), i.e. the left side of Eq. (4) at r0 = -s.  We report
  d = argmax, so frame(r) ~ ref(r - d); the paper's r0 is -d.
* CC-SN sign (Eq. 6-7).  Minimising Eq. (6) minimises sum I'^2/E, so the
  method's extremum is a minimum of the Eq. (7) correlation.  We use
  B = -1/(E + eps), turning it into a maximum.  E in Eq. (5) is the mean of
  the offset image, hence E + eps.
* Nyquist bin (even N): phi_{N/2}(s) = cos(pi s), which makes C(s) real
  and equal to the correlation at integer s.
* Grid: M = ceil(1.5 u) points per axis, centre index c = floor(M/2), grid
  offsets (m - c)/u, so the integer peak is a grid point.
* Ties: lowest row-major index, for the integer peak and the grid.
* Signed lag range [-N/2, N/2).
* Refinement: Newton on C(s) from d_grid, with fallback to d_grid when the
  Hessian is not negative definite, a step exceeds 1/u, or the result
  leaves the 0.75-px half window.
* Reference updates (Eq. 8-9): the reference E is the mean image of the
  frames (Eq. 5 makes E the mean of the frames; the substitution rule of
  Sec. III applies to the correlation, not to this average), in both CC-U
  and CC-SN.  A frame shifted back by its displacement d is I(r + d) (the
  paper's I(r - r0)); its spectrum is F[I](k) phi_ky(d_y) phi_kx(d_x) with
  the same Nyquist rule, i.e. the band-limited shift.  Frames whose
  tracking was non-finite or flat are left out of the mean.
"""
from __future__ import annotations

import math

import numpy as np

# status bits of a result (same meaning as the library's)
NONFINITE = 1
FLAT = 2
NEAR_TIE = 4
NEWTON_FALLBACK = 8
WINDOW_EXIT = 16

MODE_CCU = 0
MODE_CCSN = 1

NEAR_TIE_REL = 1e-5
NEWTON_TOL = 1e-13
NEWTON_MAX_IT = 20
HALF_WINDOW = 0.75


# --------------------------------------------------------------------------
# O1  weights (Sec. II Eq. 2-7; Sec. III substitution I -> I'^2, E -> 1/E)
# --------------------------------------------------------------------------
def weights(frame, ref, mode=MODE_CCU, eps=200.0):
    """Return (A, B): the two images whose circular cross-correlation is
    maximised.  CC-U (Eq. 4): A = I, B = E.  CC-SN (Eq. 7): A = (I+eps)^2,
    B = -1/(E+eps) (sign: the CC-SN extremum of Eq. 6 is a minimum)."""
    I = np.asarray(frame, dtype=np.float64)
    E = np.asarray(ref, dtype=np.float64)
    if mode == MODE_CCU:
        return I, E
    if mode == MODE_CCSN:
        Ep = E + eps
        if np.any(Ep <= 0):
            raise ValueError("CC-SN reference needs E + eps > 0 everywhere")
        return (I + eps) ** 2, -1.0 / Ep
    raise ValueError("unknown mode")


# --------------------------------------------------------------------------
# O2, O3  cross-power spectrum and circular correlation (Eq. 4 / Eq. 7)
# --------------------------------------------------------------------------
def cross_power(A, B):
    """X = F[A] * conj(F[B]) with numpy's unnormalised forward DFT."""
    return np.fft.fft2(A) * np.conj(np.fft.fft2(B))


def correlation(X):
    """CC(s) = Re F^{-1}[X](s) = sum_r A(r+s) B(r) (circular)."""
    return np.fft.ifft2(X).real


def direct_correlation(A, B):
    """Brute-force circular correlation sum_r A(r+s) B(r) for every lag s.
    O(N^4); for tiny images only (the FFT route must agree with it)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    ny, nx = A.shape
    out = np.zeros((ny, nx))
    for sy in range(ny):
        for sx in range(nx):
            acc = 0.0
            for y in range(ny):
                for x in range(nx):
                    acc += A[(y + sy) % ny, (x + sx) % nx] * B[y, x]
            out[sy, sx] = acc
    return out


# --------------------------------------------------------------------------
# O4  integer peak (Sec. III, first paragraph)
# --------------------------------------------------------------------------
def _signed(i, n):
    # lags s >= n/2 (ceil for odd n) map to s - n
    return i - n if 2 * i >= n else i


def integer_peak(cc):
    """Argmax of the correlation with ties to the lowest row-major index.
    Returns ((py, px) signed lags, value, flat index)."""
    flat = int(np.argmax(cc))  # numpy returns the first maximum
    ny, nx = cc.shape
    iy, ix = divmod(flat, nx)
    return (_signed(iy, ny), _signed(ix, nx)), float(cc.flat[flat]), flat


def is_near_tie(cc, rel=NEAR_TIE_REL):
    """True when the two largest correlation values are within rel*|max|."""
    v = np.sort(cc.ravel())
    return bool(v[-1] - v[-2] <= rel * abs(v[-1]))


# --------------------------------------------------------------------------
# O5  band-limited correlation and its derivatives
# --------------------------------------------------------------------------
def signed_freq(n):
    """Signed frequency index for each DFT bin k = 0..n-1."""
    return np.fft.fftfreq(n) * n


def phi(n, s, order=0):
    """Basis phi_k(s) for all k = 0..n-1 and its s-derivatives.

    phi_k(s) = exp(2 pi i k~ s / n) for the signed frequency k~, except the
    Nyquist bin of even n where phi = cos(pi s)."""
    k = signed_freq(n)
    w = 2.0 * np.pi * k / n
    v = np.exp(1j * w * s) * (1j * w) ** order
    if n % 2 == 0:
        h = n // 2
        if order == 0:
            v[h] = math.cos(math.pi * s)
        elif order == 1:
            v[h] = -math.pi * math.sin(math.pi * s)
        elif order == 2:
            v[h] = -(math.pi ** 2) * math.cos(math.pi * s)
        else:
            raise ValueError("order <= 2")
    return v


def bandlimited(X, s, dy=0, dx=0):
    """d^(dy+dx) C / ds_y^dy ds_x^dx at s = (s_y, s_x), where
    C(s) = 1/(ny nx) sum_k X(k) phi_ky(s_y) phi_kx(s_x)."""
    ny, nx = X.shape
    vy = phi(ny, s[0], dy)
    vx = phi(nx, s[1], dx)
    return float((vy @ X @ vx).real) / (ny * nx)


def gradient_hessian(X, s):
    """(C, g, H) of the band-limited correlation at s."""
    c = bandlimited(X, s)
    g = np.array([bandlimited(X, s, 1, 0), bandlimited(X, s, 0, 1)])
    hyy = bandlimited(X, s, 2, 0)
    hxx = bandlimited(X, s, 0, 2)
    hxy = bandlimited(X, s, 1, 1)
    H = np.array([[hyy, hxy], [hxy, hxx]])
    return c, g, H


# --------------------------------------------------------------------------
# O6  upsampled grid (Sec. III, first paragraph; matrix DFT after [27])
# --------------------------------------------------------------------------
def grid_size(u):
    """M = ceil(1.5 u) samples per axis, centre index c = floor(M / 2)."""
    m = int(math.ceil(1.5 * u - 1e-12))
    return m, m // 2


def grid_offsets(u):
    m, c = grid_size(u)
    return (np.arange(m) - c) / u


def upsampled_grid(X, p, u):
    """U[my, mx] = C(p + (delta_my, delta_mx)) on the 1.5-px window,
    computed as K_y X K_x^T with K[m, k] = phi_k(p + delta_m)."""
    ny, nx = X.shape
    off = grid_offsets(u)
    Ky = np.stack([phi(ny, p[0] + o) for o in off])
    Kx = np.stack([phi(nx, p[1] + o) for o in off])
    U = (Ky @ X @ Kx.T).real / (ny * nx)
    return U


def grid_peak(U, p, u):
    """Argmax of U (ties to lowest row-major index) -> d_grid."""
    m, c = grid_size(u)
    flat = int(np.argmax(U))
    my, mx = divmod(flat, U.shape[1])
    return np.array([p[0] + (my - c) / u, p[1] + (mx - c) / u]), (my, mx)


# --------------------------------------------------------------------------
# O7  Newton refinement of the maximiser of C(s)
# --------------------------------------------------------------------------
def newton(X, seed, p, u, max_it=NEWTON_MAX_IT, tol=NEWTON_TOL):
    """Newton iterations on C from `seed`.  Returns (d_hat, C(d_hat), H, status).
    Falls back to the seed when H is not negative definite or a step is
    longer than 1/u; flags a window exit when |d_hat - p|_inf > 0.75."""
    s = np.array(seed, dtype=np.float64)
    status = 0
    for _ in range(max_it):
        _, g, H = gradient_hessian(X, s)
        if not (H[0, 0] < 0 and np.linalg.det(H) > 0):
            status |= NEWTON_FALLBACK
            s = np.array(seed, dtype=np.float64)
            break
        step = -np.linalg.solve(H, g)
        if np.max(np.abs(step)) > 1.0 / u:
            status |= NEWTON_FALLBACK
            s = np.array(seed, dtype=np.float64)
            break
        s = s + step
        if np.max(np.abs(step)) < tol:
            break
    if np.max(np.abs(s - np.asarray(p, dtype=np.float64))) > HALF_WINDOW:
        status |= WINDOW_EXIT
        s = np.array(seed, dtype=np.float64)
    c, _, H = gradient_hessian(X, s)
    return s, c, H, status


# --------------------------------------------------------------------------
# the whole per-frame path
# --------------------------------------------------------------------------
def track(frame, ref, u, mode=MODE_CCU, eps=200.0, newton_it=NEWTON_MAX_IT):
    """Displacement of `frame` relative to `ref` (frame(r) ~ ref(r - d)).

    Returns a dict with d (Newton maximiser), d_grid (the paper's upsampled
    estimate), p (integer peak lag), peak (C(d)), hess (H at d, [yy, yx, xx]),
    cc_peak (integer-lag correlation maximum), status bits."""
    I = np.asarray(frame, dtype=np.float64)
    out = dict(d=np.full(2, np.nan), d_grid=np.full(2, np.nan), p=(0, 0),
               peak=np.nan, hess=np.full(3, np.nan), cc_peak=np.nan, status=0)
    if not np.all(np.isfinite(I)):
        out["status"] = NONFINITE
        return out
    A, B = weights(I, ref, mode, eps)
    if A.max() == A.min():
        out.update(status=FLAT, d=np.zeros(2), d_grid=np.zeros(2), peak=0.0,
                   hess=np.zeros(3), cc_peak=0.0)
        return out
    X = cross_power(A, B)
    cc = correlation(X)
    p, ccp, _ = integer_peak(cc)
    status = NEAR_TIE if is_near_tie(cc) else 0
    U = upsampled_grid(X, p, u)
    d_grid, m = grid_peak(U, p, u)
    d, c, H, st = newton(X, d_grid, p, u, max_it=newton_it)
    out.update(d=d, d_grid=d_grid, p=p, peak=c, hess=np.array([H[0, 0], H[0, 1], H[1, 1]]),
               cc_peak=ccp, status=status | st, grid_index=m)
    # diagnostics for comparisons made in lower precision (no part of the
    # result): the gaps between the two largest correlation and grid values,
    # and the grid maximum without the DC term's constant X(0)/(ny nx)
    top_cc = np.sort(cc.ravel())[-2:]
    top_u = np.sort(U.ravel())[-2:]
    out.update(cc_gap=float(top_cc[1] - top_cc[0]), grid_gap=float(top_u[1] - top_u[0]),
               grid_ac=float(abs(top_u[1] - X[0, 0].real / X.size)))
    return out


def track_many(frames, refs, ref_ids, u, mode=MODE_CCU, eps=200.0):
    """track() over a list of frames; returns stacked arrays."""
    res = [track(f, refs[int(r)], u, mode, eps) for f, r in zip(frames, ref_ids)]
    return dict(
        d=np.array([r["d"] for r in res]),
        d_grid=np.array([r["d_grid"] for r in res]),
        p=np.array([r["p"] for r in res], dtype=np.int64),
        peak=np.array([r["peak"] for r in res]),
        hess=np.array([r["hess"] for r in res]),
        status=np.array([r["status"] for r in res], dtype=np.int64),
    )


# --------------------------------------------------------------------------
# O8  adjoint of (d_hat, C(d_hat)) by the implicit function theorem
# --------------------------------------------------------------------------
def _shift_kernel(shape, s, lam, cbar):
    """Psi(k) = (1/(ny nx)) * (lam_y d/ds_y + lam_x d/ds_x + cbar) phi_k(s)
    on the full 2-D spectrum."""
    ny, nx = shape
    vy0, vy1 = phi(ny, s[0], 0), phi(ny, s[0], 1)
    vx0, vx1 = phi(nx, s[1], 0), phi(nx, s[1], 1)
    psi = (lam[0] * np.outer(vy1, vx0) + lam[1] * np.outer(vy0, vx1)
           + cbar * np.outer(vy0, vx0))
    return psi / (ny * nx)


def adjoint(frame, ref, fwd, g_d, g_peak=0.0, mode=MODE_CCU, eps=200.0):
    """Gradients of L = g_d . d_hat + g_peak * C(d_hat) with respect to the
    frame I and the reference E.

    At the maximiser grad_s C = 0, so d d_hat / dtheta = -H^{-1} d(grad_s C)/dtheta
    and dC(d_hat)/dtheta = dC/dtheta.  With lam = -H^{-1} g_d:
        dL/dA(x) = sum_k conj(F[B](k)) Psi(k) exp(-2 pi i k.x / N)
        dL/dB(x) = sum_k F[A](k)       Psi(k) exp(+2 pi i k.x / N)
    where Psi = (lam . grad_s + g_peak) phi_k(s) / (ny nx) at s = d_hat.
    CC-SN chains through A = (I+eps)^2 and B = -1/(E+eps)."""
    if fwd["status"] & (NONFINITE | FLAT | NEWTON_FALLBACK | WINDOW_EXIT):
        z = np.zeros(np.shape(frame))
        return z, z.copy()
    I = np.asarray(frame, dtype=np.float64)
    A, B = weights(I, ref, mode, eps)
    h = fwd["hess"]
    H = np.array([[h[0], h[1]], [h[1], h[2]]])
    lam = -np.linalg.solve(H, np.asarray(g_d, dtype=np.float64))
    psi = _shift_kernel(A.shape, fwd["d"], lam, g_peak)
    ny, nx = A.shape
    FA = np.fft.fft2(A)
    FB = np.fft.fft2(B)
    gA = np.fft.fft2(np.conj(FB) * psi).real
    gB = (np.fft.ifft2(FA * psi) * (ny * nx)).real
    if mode == MODE_CCU:
        return gA, gB
    E = np.asarray(ref, dtype=np.float64)
    return gA * 2.0 * (I + eps), gB / (E + eps) ** 2


# --------------------------------------------------------------------------
# O9  Fisher information and Cramer-Rao bound of the displacement
# --------------------------------------------------------------------------
def derivative_images(mu):
    """d mu / d d_j for mu(r; d) = mu~(r - d) at d = 0, where mu~ is the
    band-limited (trigonometric) interpolant of the sampled mean image.
    Returns [d/d d_y, d/d d_x].  The Nyquist derivative is zero under the
    cos(pi s) convention at s = 0."""
    mu = np.asarray(mu, dtype=np.float64)
    ny, nx = mu.shape
    F = np.fft.fft2(mu)
    vy = phi(ny, 0.0, 1)
    vx = phi(nx, 0.0, 1)
    # mu~(r - d) = (1/N) sum_k F(k) phi_k(r - d); d/dd_j = -(1/N) sum F dphi
    dy = -np.fft.ifft2(F * vy[:, None]).real
    dx = -np.fft.ifft2(F * vx[None, :]).real
    return dy, dx


def fisher(mu):
    """Poisson Fisher matrix F_jl = sum_r (d_j mu)(d_l mu) / mu."""
    mu = np.asarray(mu, dtype=np.float64)
    dy, dx = derivative_images(mu)
    w = 1.0 / mu
    return np.array([[np.sum(dy * dy * w), np.sum(dy * dx * w)],
                     [np.sum(dx * dy * w), np.sum(dx * dx * w)]])


def crb(mu):
    """Cramer-Rao bound on the displacement covariance: F^{-1}."""
    return np.linalg.inv(fisher(mu))


def shot_noise_limit(w0, n_photons):
    """Shot-noise limit of Sec. IV: sigma_pos = w0 / (2 sqrt(N_gamma))."""
    return w0 / (2.0 * math.sqrt(n_photons))


# --------------------------------------------------------------------------
# O10  offline reference (Sec. III.A, Eq. 8)
# --------------------------------------------------------------------------
def align_spectrum(F, d):
    """Spectrum of a frame shifted back by its displacement d = (d_y, d_x):
    F[I(r + d)](k) = F[I](k) phi_ky(d_y) phi_kx(d_x) (band-limited shift,
    Nyquist bins scaled by cos(pi d))."""
    ny, nx = F.shape
    return F * np.outer(phi(ny, d[0]), phi(nx, d[1]))


def mean_aligned(frames, ds, statuses=None):
    """Eq. (8) for one pass: the inverse transform of (1/n) sum_i
    F[I_i(r - r0_i)] over the frames that tracked (status without NONFINITE
    or FLAT), with r0 = -d."""
    acc = None
    n = 0
    for i, (f, d) in enumerate(zip(frames, ds)):
        if statuses is not None and (int(statuses[i]) & (NONFINITE | FLAT)):
            continue
        a = align_spectrum(np.fft.fft2(np.asarray(f, dtype=np.float64)), d)
        acc = a if acc is None else acc + a
        n += 1
    if n == 0:
        raise ValueError("no frame to average")
    return np.fft.ifft2(acc / n).real


def iterative_reference(frames, u, passes, mode=MODE_CCU, eps=200.0):
    """Sec. III.A: E_0 = I_0; pass n tracks every frame against E_{n-1} and
    E_n = mean_aligned(frames, displacements).  Returns (E_passes, the
    results of the last pass)."""
    E = np.asarray(frames[0], dtype=np.float64)
    res = None
    for _ in range(passes):
        res = [track(f, E, u, mode, eps) for f in frames]
        E = mean_aligned(frames, [r["d"] for r in res], [r["status"] for r in res])
    return E, res


# --------------------------------------------------------------------------
# O11  real-time reference (Sec. III.B, Eq. 9)
# --------------------------------------------------------------------------
def realtime_track(frames, u, a0, mode=MODE_CCU, eps=200.0):
    """Tracks the frames in order against a reference updated after each
    frame by F[E_i] = a0 F[I_i(r - r0_i)] + b1 F[E_{i-1}], b1 = 1 - a0,
    starting from E_{-1} = E_0 = I_0 (so frame 0 is tracked against itself
    and leaves E unchanged).  A frame that did not track (NONFINITE or FLAT)
    leaves the reference unchanged.  Returns the list of results."""
    E = np.asarray(frames[0], dtype=np.float64)
    FE = np.fft.fft2(E)
    b1 = 1.0 - a0
    out = []
    for f in frames:
        r = track(f, E, u, mode, eps)
        out.append(r)
        if r["status"] & (NONFINITE | FLAT):
            continue
        FE = a0 * align_spectrum(np.fft.fft2(np.asarray(f, dtype=np.float64)), r["d"]) + b1 * FE
        E = np.fft.ifft2(FE).real
    return out


# --------------------------------------------------------------------------
# O12  drift correction (Sec. III.B, Eq. 10-12)
# --------------------------------------------------------------------------
def drift_filter(r, a0, rate_limit=0.0):
    """Offsets R_n and corrected displacements r_n - R_n for a sequence of
    displacements r ([n, 2]).  Eq. (10): R_0 = a0 r_0 and
    R_n = a0 r_n + b1 R_{n-1} for n >= 1.  With rate_limit = alpha/u > 0,
    Eq. (11)-(12) replace the update from n = 1 on:
    dR_n = a0 r_n + (b1 - 1) R_{n-1}, and a step longer than rate_limit is
    cut to that length along dR_n.  The first offset is Eq. (10)'s R_0 in
    both forms (the rate limit acts on steps between offsets)."""
    r = np.asarray(r, dtype=np.float64)
    b1 = 1.0 - a0
    R = np.zeros(2)
    offsets = np.zeros_like(r)
    for n, rn in enumerate(r):
        if n == 0:
            R = a0 * rn
        elif rate_limit > 0.0:
            dR = a0 * rn + (b1 - 1.0) * R
            L = math.hypot(dR[0], dR[1])
            R = R + (rate_limit * dR / L if L > rate_limit else dR)
        else:
            R = a0 * rn + b1 * R
        offsets[n] = R
    return offsets, r - offsets
