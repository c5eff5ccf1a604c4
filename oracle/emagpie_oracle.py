"""FP64 CPU oracle of the eMAGPIE stochastic surrogate-minimisation epoch.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the HIP path is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the HIP library: the two
meet only in the seeded inputs they are both handed.

Everything is complex128 / float64.  Each function cites the passage of the
paper (arXiv 2511.01793, "Stochastic Multigrid Method for Blind
Ptychographic Phase Retrieval") it follows.  Where the paper is silent the
reading taken is stated in the docstring:

* F is the unnormalised 2-D DFT and F^-1 carries 1/m^2 (fixed by the dp_avg
  rule of Sec. 4.1 reproducing ||Q||);
* theta(0) := 0 (footnote of Def. 2.1);
* patches are integer top-left windows, 0 <= row, col <= n - m;
* I_h^H is 2x2 mean pooling and I_H^h the piecewise-constant copy (the
  non-negative disjoint restriction with I_h^H I_H^h = I, I_H^h = 4 I_h^H^T);
* three or more levels apply the two-level construction recursively;
* a minibatch uses the state at its start for every member; the object and
  probe one-variable steps are the exact minimisers of the summed
  regularised surrogates; the joint step is taken once per pixel after that;
* zero denominators keep the old value;
* the scan order is a Fisher-Yates shuffle driven by SplitMix64.

Parity status: every function below is pinned by a CPU test except the
multi-epoch trajectory, which the paper prints no values for (it is pinned
only GPU-against-oracle from identical state).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


# --------------------------------------------------------------------------
# Fourier transform and patch operator (Sec. 2.1)
# --------------------------------------------------------------------------

def dft2(psi: np.ndarray) -> np.ndarray:
    """Unnormalised 2-D DFT F over the last two axes (Sec. 2.1)."""
    return np.fft.fft2(np.asarray(psi, dtype=np.complex128), axes=(-2, -1))


def idft2(Psi: np.ndarray) -> np.ndarray:
    """Inverse of dft2, carrying the 1/m^2 factor."""
    return np.fft.ifft2(np.asarray(Psi, dtype=np.complex128), axes=(-2, -1))


def patch(z: np.ndarray, pos, m: int) -> np.ndarray:
    """z_k = P_k z: the m x m window with top-left corner pos (Sec. 2.1, Def. 2.1)."""
    r, c = int(pos[0]), int(pos[1])
    if r < 0 or c < 0 or r + m > z.shape[0] or c + m > z.shape[1]:
        raise ValueError("scan position outside the object")
    return z[r:r + m, c:c + m]


# --------------------------------------------------------------------------
# Revised exit wave, misfit, gradients (Def. 2.1, Eq. 1, Sec. 2.1)
# --------------------------------------------------------------------------

def unit_phase(Psi: np.ndarray) -> np.ndarray:
    """exp(i theta(Psi)) with theta(0) = 0 (footnote of Def. 2.1)."""
    mag = np.abs(Psi)
    out = np.ones_like(Psi, dtype=np.complex128)
    nz = mag > 0
    out[nz] = Psi[nz] / mag[nz]
    return out


def amplitudes(d: np.ndarray) -> np.ndarray:
    """sqrt(d) of Def. 2.1; negative counts are clamped to zero."""
    d = np.asarray(d, dtype=np.float64)
    if not np.all(np.isfinite(d)):
        raise ValueError("non-finite intensity")
    return np.sqrt(np.maximum(d, 0.0))


def revised_exit_wave(Q: np.ndarray, zk: np.ndarray, ak: np.ndarray,
                      prev_phase: np.ndarray | None = None) -> np.ndarray:
    """R_k(Q, z_k) = F^-1( sqrt(d_k) . exp(i theta(F(Q . z_k))) ) (Def. 2.1).

    prev_phase (optional, m x m unit phasors exp(i theta)): the stateful rule stated after
    Eq. 3 -- where F(Q . z_k) is zero, theta is the phase pattern k had at the previous
    iterate (0 at the first).  Without it theta(0) = 0 (footnote of Def. 2.1).
    """
    return idft2(ak * phase_used(dft2(Q * zk), prev_phase))


def phase_used(Psi: np.ndarray, prev_phase: np.ndarray | None) -> np.ndarray:
    """exp(i theta) of Psi, with the zero bins taking prev_phase (or 1 when it is None)."""
    u = unit_phase(Psi)
    if prev_phase is not None:
        zero = np.abs(Psi) == 0
        u[zero] = prev_phase[zero]
    return u


def misfit_terms(Q, z, positions, a) -> np.ndarray:
    """Phi_k = 1/2 ||Q . P_k z - R_k(Q, P_k z)||^2 for every k (Eq. 1)."""
    m = Q.shape[0]
    out = np.empty(len(positions))
    for k, p in enumerate(positions):
        zk = patch(z, p, m)
        r = Q * zk - revised_exit_wave(Q, zk, a[k])
        out[k] = 0.5 * float(np.vdot(r, r).real)
    return out


def misfit(Q, z, positions, a) -> float:
    """Exit-wave misfit Phi(Q, z) of Eq. 1 (real-space form)."""
    return float(misfit_terms(Q, z, positions, a).sum())


def gradients(Q, z, positions, a):
    """CR-calculus gradients of Phi (Sec. 2.1), gradient = d/dx + i d/dy.

    grad_z Phi = sum_k P_k^T [conj(Q) . (Q . z_k - R_k)],
    grad_Q Phi = sum_k conj(z_k) . (Q . z_k - R_k).
    Returns (grad_z, grad_Q, Phi).
    """
    m = Q.shape[0]
    gz = np.zeros_like(z, dtype=np.complex128)
    gq = np.zeros_like(Q, dtype=np.complex128)
    phi = 0.0
    for k, p in enumerate(positions):
        r0, c0 = int(p[0]), int(p[1])
        zk = patch(z, p, m)
        e = Q * zk - revised_exit_wave(Q, zk, a[k])
        gz[r0:r0 + m, c0:c0 + m] += np.conj(Q) * e
        gq += np.conj(zk) * e
        phi += 0.5 * float(np.vdot(e, e).real)
    return gz, gq, phi


def surrogate(Q, z, positions, R_frozen) -> float:
    """Quadratic surrogate of Eq. 3 with the revised exit waves frozen at iterate j."""
    m = Q.shape[0]
    tot = 0.0
    for k, p in enumerate(positions):
        r = Q * patch(z, p, m) - R_frozen[k]
        tot += 0.5 * float(np.vdot(r, r).real)
    return tot


# --------------------------------------------------------------------------
# Regularisers (Sec. 2.2 and Sec. 4)
# --------------------------------------------------------------------------

def probe_regulariser(Q: np.ndarray, alpha: float) -> np.ndarray:
    """u_Q(Q) = alpha (||Q||_inf^2 - |Q|^2); it regularises the object step (Sec. 2.2, Sec. 4)."""
    q2 = np.abs(Q) ** 2
    return alpha * (q2.max() - q2)


def patch_regulariser(zk: np.ndarray, alpha_z: float) -> np.ndarray:
    """u_z(z_k) = alpha_z (||z_k||_inf^2 - |z_k|^2); it regularises the probe step.

    The sup norm is taken over patch k (Sec. 4 writes ||z_k^(j)||_inf); alpha_z = 1 is the
    ePIE probe step used in all experiments.
    """
    z2 = np.abs(zk) ** 2
    return alpha_z * (z2.max() - z2)


# --------------------------------------------------------------------------
# Multigrid object step (Sec. 3.2, Eqs. 12-15)
# --------------------------------------------------------------------------

def restrict(x: np.ndarray) -> np.ndarray:
    """I_h^H: 2x2 mean pooling on the patch-local grid (Sec. 3.2)."""
    h, w = x.shape
    return 0.25 * (x[0::2, 0::2] + x[1::2, 0::2] + x[0::2, 1::2] + x[1::2, 1::2])


def prolong(x: np.ndarray) -> np.ndarray:
    """I_H^h = 4 (I_h^H)^T: copy each coarse value to its 2x2 children (Sec. 3.2)."""
    return np.repeat(np.repeat(x, 2, axis=0), 2, axis=1)


def _safe_div(num, den):
    out = np.zeros(np.broadcast(num, den).shape, dtype=np.result_type(num, den, np.float64))
    nz = den != 0
    out[nz] = (np.broadcast_to(num, out.shape)[nz] / np.broadcast_to(den, out.shape)[nz])
    return out


def mg_weights(Q: np.ndarray):
    """Interlevel weights of Eq. 14.

    W_z = |Q|^2 / (I_H^h I_h^H |Q|^2), W_R = (I_H^h Q_H) . W_z / Q, W_u^H = |Q_H|^2 / (I_h^H |Q|^2).
    W_R is evaluated as (I_H^h Q_H) . conj(Q) / (I_H^h I_h^H |Q|^2), equal to the printed form
    wherever Q != 0 and its continuous extension where Q = 0; weights over a block on which
    Q vanishes identically are set to 0.
    """
    q2 = np.abs(Q) ** 2
    rq2 = restrict(q2)
    QH = restrict(Q)
    Wz = _safe_div(q2, prolong(rq2))
    WR = _safe_div(prolong(QH) * np.conj(Q), prolong(rq2))
    Wu = _safe_div(np.abs(QH) ** 2, rq2)
    return Wz, WR, Wu


def magpie_coarse_correction(Q, zk, Rk, u, levels: int) -> np.ndarray:
    """I_H^h (z^_H - z_H): the coarse-grid correction of the MAGPIE object step (Sec. 3.2).

    Restricted terms follow Eq. 15 with the weights of Eq. 14; the coarse problem is solved in
    closed form by the same (recursive) MAGPIE step.  With levels == 2 that step is exactly the
    printed coarse update z^_H = z_H + conj(Q_H)(R_H - Q_H z_H)/(u_H + |Q_H|^2); more levels
    treat the coarse problem as the fine level of the next pair.  R_H is the restricted term of
    Eq. 15 (no coarse Fourier transform).  Where the coarse denominator u_H + |Q_H|^2 vanishes on
    a block, the block takes its continuous extension sum(conj(Q)(R - Q z))/sum(u + |Q|^2)
    (zero if that denominator vanishes too).
    """
    if levels <= 1:
        return np.zeros_like(zk, dtype=np.complex128)
    Wz, WR, Wu = mg_weights(Q)
    QH = restrict(Q)
    zH = restrict(Wz * zk)
    RH = restrict(WR * Rk)
    uH = Wu * restrict(u)
    zH_hat = magpie_object_step(QH, zH, RH, uH, levels - 1)
    den = uH + np.abs(QH) ** 2
    bad = den == 0
    if np.any(bad):
        g = np.conj(Q) * (Rk - Q * zk)
        ext = _safe_div(restrict(g), restrict(u + np.abs(Q) ** 2))
        zH_hat = np.where(bad, zH + ext, zH_hat)
    return prolong(zH_hat - zH)


def magpie_object_step(Q, zk, Rk, u, levels: int) -> np.ndarray:
    """MAGPIE object minimiser z^+_k (Sec. 3.2, closed forms after Eq. 15).

    z'_k = z_k + I_H^h (z^_H - z_H);  z^+_k = z'_k + conj(Q)(R_k - Q z'_k)/(u + |Q|^2).
    With levels == 1 this is the regularised one-variable step of Eq. 7 / Eq. 9.  A pixel with a
    zero denominator keeps z'_k.
    """
    zprime = zk + magpie_coarse_correction(Q, zk, Rk, u, levels)
    den = u + np.abs(Q) ** 2
    return zprime + _safe_div(np.conj(Q) * (Rk - Q * zprime), den)


def probe_step_single(Q, zk, Rk, alpha_z: float) -> np.ndarray:
    """Q^+ = Q + conj(z_k)(R_k - Q z_k)/(|z_k|^2 + u_z) (Eq. 8 / Eq. 9)."""
    uz = patch_regulariser(zk, alpha_z)
    den = np.abs(zk) ** 2 + uz
    return Q + _safe_div(np.conj(zk) * (Rk - Q * zk), den)


# --------------------------------------------------------------------------
# Geometric-mean, phase-aligned joint step (Eq. 6)
# --------------------------------------------------------------------------

def aligned_sqrt(x: np.ndarray, xplus: np.ndarray) -> np.ndarray:
    """x~ with x~^2 = x . x^+ and |arg(x~ conj(x))| <= pi/2 (Eq. 6).

    The principal root is taken and negated when Re(root . conj(x)) < 0; at a tie (= 0) the
    principal root is kept.  x = 0 gives 0.
    """
    s = np.sqrt(np.asarray(x, np.complex128) * np.asarray(xplus, np.complex128))
    flip = (s * np.conj(x)).real < 0
    return np.where(flip, -s, s)


# --------------------------------------------------------------------------
# One minibatch step (Sec. 3, Prop. 3.2, Sec. 3.2; minibatch reading in the header)
# --------------------------------------------------------------------------

def step_minibatch(Q, z, positions, a, idx, *, alpha: float, alpha_z: float = 1.0,
                   levels: int = 1, update_probe: bool = True, joint: bool = True,
                   phase_mem: np.ndarray | None = None):
    """Apply one eMAGPIE minibatch update to (Q, z) and return the new state.

    For the members k of idx, all evaluated at the state at the start of the batch:
      R_k = revised exit wave (Def. 2.1), u = u_Q(Q) (Sec. 4),
      z'_k = z_k + MAGPIE coarse correction (Sec. 3.2),
      object: z^+ = argmin_z sum_k [Phi~_k(Q, P_k z) + 1/2 <u, |P_k z - z'_k|^2>]
              = sum_k P_k^T (conj(Q) R_k + u z'_k) / sum_k P_k^T (|Q|^2 + u) on touched pixels,
      probe:  Q^+ = argmin_Q sum_k [Phi~_k(Q, z_k) + 1/2 <u_z(z_k), |Q - Q^(j)|^2>]
              = sum_k (conj(z_k) R_k + u_z,k Q) / sum_k (|z_k|^2 + u_z,k)   (Eq. 8),
      joint:  z <- aligned_sqrt(z, z^+), Q <- aligned_sqrt(Q, Q^+)  (Eq. 6).
    With one member and one level this is the step of Prop. 3.2 (Eqs. 6-9); joint=False gives
    the rPIE update of Eq. 2.  phase_mem (optional, N x m x m unit phasors, updated in place):
    the stateful zero-bin phase rule stated after Eq. 3; each member reads its previous phases
    and stores the ones it used.  Returns (Q_new, z_new, info) with info holding z^+, Q^+, the
    touched mask, the revised waves and the sampled misfit sum_k Phi_k.
    """
    Q = np.asarray(Q, np.complex128)
    z = np.asarray(z, np.complex128)
    m = Q.shape[0]
    u = probe_regulariser(Q, alpha)
    D = np.abs(Q) ** 2 + u
    Nacc = np.zeros_like(z)
    Dacc = np.zeros(z.shape)
    Macc = np.zeros_like(Q)
    Eacc = np.zeros(Q.shape)
    Rs = []
    phi = 0.0
    for k in idx:
        p = positions[k]
        r0, c0 = int(p[0]), int(p[1])
        zk = patch(z, p, m).copy()
        if phase_mem is None:
            Rk = revised_exit_wave(Q, zk, a[k])
        else:
            ph = phase_used(dft2(Q * zk), phase_mem[k])
            Rk = idft2(a[k] * ph)
            phase_mem[k] = ph
        Rs.append(Rk)
        e = Q * zk - Rk
        phi += 0.5 * float(np.vdot(e, e).real)
        zprime = zk + magpie_coarse_correction(Q, zk, Rk, u, levels)
        Nacc[r0:r0 + m, c0:c0 + m] += np.conj(Q) * Rk + u * zprime
        Dacc[r0:r0 + m, c0:c0 + m] += D
        uz = patch_regulariser(zk, alpha_z)
        Macc += np.conj(zk) * Rk + uz * Q
        Eacc += np.abs(zk) ** 2 + uz
    touched = Dacc > 0
    zplus = z.copy()
    zplus[touched] = Nacc[touched] / Dacc[touched]
    z_new = aligned_sqrt(z, zplus) if joint else zplus
    z_new = np.where(touched, z_new, z)
    if update_probe:
        okq = Eacc > 0
        Qplus = Q.copy()
        Qplus[okq] = Macc[okq] / Eacc[okq]
        Q_new = aligned_sqrt(Q, Qplus) if joint else Qplus
    else:
        Qplus = Q.copy()
        Q_new = Q.copy()
    info = dict(zplus=zplus, Qplus=Qplus, touched=touched, R=Rs, sampled_misfit=phi)
    return Q_new, z_new, info


# --------------------------------------------------------------------------
# Scan order (Sec. 2.2: random permutation every iteration)
# --------------------------------------------------------------------------

class SplitMix64:
    """Vigna's SplitMix64 generator (public-domain reference definition)."""

    def __init__(self, state: int):
        self.state = state & MASK64

    def next(self) -> int:
        self.state = (self.state + GOLDEN_GAMMA) & MASK64
        x = self.state
        x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & MASK64
        return x ^ (x >> 31)


def permutation(seed: int, epoch: int, n: int) -> np.ndarray:
    """Random scan order of one sweep: Durstenfeld's Fisher-Yates shuffle of 0..n-1.

    The generator for sweep e starts from state seed XOR (e * 0x9E3779B97F4A7C15) mod 2^64;
    the swap partner of slot i is floor(x * (i + 1) / 2^64) for the next 64-bit output x.
    """
    g = SplitMix64((seed ^ ((epoch * GOLDEN_GAMMA) & MASK64)) & MASK64)
    perm = list(range(n))
    for i in range(n - 1, 0, -1):
        j = (g.next() * (i + 1)) >> 64
        perm[i], perm[j] = perm[j], perm[i]
    return np.asarray(perm, dtype=np.int32)


def run_epoch(Q, z, positions, a, *, seed: int, epoch: int, minibatch: int, alpha: float,
              alpha_z: float = 1.0, levels: int = 1, update_probe: bool = True,
              perm: np.ndarray | None = None, joint: bool = True,
              phase_mem: np.ndarray | None = None):
    """One sweep (iteration j) over all scan positions in random order, in consecutive
    minibatches; the last one may be short (Sec. 3, stochastic strategy).  Returns (Q, z, sampled)."""
    n_pos = len(positions)
    order = permutation(seed, epoch, n_pos) if perm is None else np.asarray(perm)
    sampled = 0.0
    for s in range(0, n_pos, minibatch):
        Q, z, info = step_minibatch(Q, z, positions, a, order[s:s + minibatch], alpha=alpha,
                                    alpha_z=alpha_z, levels=levels, update_probe=update_probe,
                                    joint=joint, phase_mem=phase_mem)
        sampled += info["sampled_misfit"]
    return Q, z, sampled


# --------------------------------------------------------------------------
# Initialisation (Sec. 4.1)
# --------------------------------------------------------------------------

def dp_avg(d: np.ndarray) -> float:
    """dp_avg = sqrt(sum_ij mean_k d_k,ij) / m (Sec. 4.1)."""
    d = np.asarray(d, dtype=np.float64)
    m = d.shape[-1]
    return float(np.sqrt(d.mean(axis=0).sum()) / m)


def normalise_probe(Q0: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Q0 <- Q0 . dp_avg / ||Q0||_2 (Sec. 4.1)."""
    Q0 = np.asarray(Q0, np.complex128)
    return Q0 * (dp_avg(d) / np.linalg.norm(Q0))
