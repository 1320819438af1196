"""Other PM time-stepping schemes than FastPM's (float64).

Test infrastructure: see the package docstring.

Section 2 of the paper builds on the FastPM kick and drift operators and
notes that other PM schemes could be put in the same framework; it defines
none.  Two readings are implemented, both as kick-drift-kick leapfrogs over
the same scale factors and the same PM force as ``pm.kdk_run``:

* ``leapfrog_run``: the standard symplectic leapfrog of the equations of
  motion dx/da = p / (a^3 E), dp/da = F / (a^2 E), with the kick and drift
  factors the plain time integrals of those right-hand sides,
      K(ai -> aj) = int_ai^aj da / (a^2 E(a)),
      D(ai -> aj) = int_ai^aj da / (a^3 E(a)),
  i.e. the force and momentum held constant over each (half) step, instead
  of FastPM's factors that make the linear growing mode exact.

* ``cola_run``: the leapfrog above applied in the frame that moves with the
  particles' LPT trajectory (the comoving-Lagrangian-acceleration idea of
  Tassev, Zaldarriaga & Eisenstein 2013).  With the LPT displacement fields
  Psi1, Psi2 of the initial conditions (mesh units, per particle),
      x_LPT(a) = q + D1(a) Psi1 + D2(a) Psi2,
      p_LPT(a) = a^3 E dx_LPT/da = a^2 E (f1 D1 Psi1 + f2 D2 Psi2),
  and, from the growth equations in a,
      a^2 E dp_LPT/da = 1.5 Omega_m [D1 Psi1 + (D2 - D1^2) Psi2] =: F_LPT(a),
  the residual r = x - x_LPT, p_r = p - p_LPT obeys
      dr/da = p_r / (a^3 E),  dp_r/da = (F(x) - F_LPT(a)) / (a^2 E),
  which is integrated by the plain leapfrog while the LPT part of every
  drift is added exactly: x += p_r D + (D1(aj) - D1(ai)) Psi1
  + (D2(aj) - D2(ai)) Psi2.  Where the PM force equals the LPT force (the
  linear regime) the residual stays zero for any step size.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad

from . import cosmology as cm
from . import pm


def std_kick(ai, aj, omega_m):
    """int_ai^aj da / (a^2 E(a)) (library quadrature)."""
    return quad(lambda a: 1.0 / (a * a * float(cm.hubble(a, omega_m))), ai, aj, epsabs=0, epsrel=1e-13)[0]


def std_drift(ai, aj, omega_m):
    """int_ai^aj da / (a^3 E(a)) (library quadrature)."""
    return quad(lambda a: 1.0 / (a ** 3 * float(cm.hubble(a, omega_m))), ai, aj, epsabs=0, epsrel=1e-13)[0]


def lpt_force_coeffs(a, omega_m):
    """(c1, c2) with F_LPT(a) = c1 Psi1 + c2 Psi2: 1.5 Om D1, 1.5 Om (D2 - D1^2)."""
    d1, _, d2, _ = (float(v[0]) for v in cm.growth(a, omega_m))
    return 1.5 * omega_m * d1, 1.5 * omega_m * (d2 - d1 * d1)


def lpt_momentum_coeffs(a, omega_m):
    """(q1, q2) with p_LPT(a) = q1 Psi1 + q2 Psi2: a^2 E f1 D1, a^2 E f2 D2."""
    d1, f1, d2, f2 = (float(v[0]) for v in cm.growth(a, omega_m))
    e = float(cm.hubble(a, omega_m))
    return a * a * e * f1 * d1, a * a * e * f2 * d2


def displacement_fields(workload, noise=None):
    """Psi1, Psi2 of the initial conditions in mesh units, [Np^3][3] in
    particle order (B times the lattice-unit fields of Gen-IC; Psi2 = 0 for
    first-order LPT)."""
    from . import lpt
    from .rng import white_noise
    if noise is None:
        noise = white_noise(workload.seed, workload.n_part)
    dk = lpt.linear_field_k(noise, workload.box_size, workload.cosmo)
    s1, s2 = lpt.lpt_displacements(dk, workload.lpt_order)
    b = workload.n_mesh // workload.n_part
    return b * s1.reshape(-1, 3), b * s2.reshape(-1, 3)


def leapfrog_run(x, p, a_list, n_mesh, n_particles, omega_m, force_fn=None, **kw):
    """Plain KDK leapfrog (factors above) from a_list[0] to a_list[-1]."""
    fn = force_fn or (lambda xx: pm.force(xx, n_mesh, n_particles, omega_m, **kw))
    x = np.array(x, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    f = fn(x)
    for ai, aj in zip(a_list[:-1], a_list[1:]):
        ac = cm.half_step(ai, aj)
        p = p + f * std_kick(ai, ac, omega_m)
        x = pm.wrap(x + p * std_drift(ai, aj, omega_m), n_mesh)
        f = fn(x)
        p = p + f * std_kick(ac, aj, omega_m)
    return x, p, f


def cola_run(x, p, psi1, psi2, a_list, n_mesh, n_particles, omega_m, force_fn=None, **kw):
    """Leapfrog of the residual from the LPT trajectory (module docstring).
    x, p: the state at a_list[0] (any state, not only the LPT one); returns
    (x, p, F) at a_list[-1] with p the full momentum."""
    fn = force_fn or (lambda xx: pm.force(xx, n_mesh, n_particles, omega_m, **kw))
    psi1 = np.asarray(psi1, dtype=np.float64)
    psi2 = np.asarray(psi2, dtype=np.float64)
    x = np.array(x, dtype=np.float64)
    a0 = a_list[0]
    q1, q2 = lpt_momentum_coeffs(a0, omega_m)
    pr = np.array(p, dtype=np.float64) - (q1 * psi1 + q2 * psi2)

    def resid_force(xx, a):
        c1, c2 = lpt_force_coeffs(a, omega_m)
        return fn(xx) - (c1 * psi1 + c2 * psi2)
    f = resid_force(x, a0)
    for ai, aj in zip(a_list[:-1], a_list[1:]):
        ac = cm.half_step(ai, aj)
        pr = pr + f * std_kick(ai, ac, omega_m)
        d1i, _, d2i, _ = (float(v[0]) for v in cm.growth(ai, omega_m))
        d1j, _, d2j, _ = (float(v[0]) for v in cm.growth(aj, omega_m))
        x = pm.wrap(x + pr * std_drift(ai, aj, omega_m) + (d1j - d1i) * psi1 + (d2j - d2i) * psi2, n_mesh)
        f = resid_force(x, aj)
        pr = pr + f * std_kick(ac, aj, omega_m)
    a1 = a_list[-1]
    q1, q2 = lpt_momentum_coeffs(a1, omega_m)
    c1, c2 = lpt_force_coeffs(a1, omega_m)
    return x, pr + q1 * psi1 + q2 * psi2, f + c1 * psi1 + c2 * psi2
