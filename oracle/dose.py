"""FP64 oracle of the dose estimate (Sec. II.H, Eqs. 6-7).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may use it; the product library never does.

The paper estimates the dose per particle at each energy from the rays of a
projection: every ray i deposits, per incident photon of energy E, the energy
E (mu_en / mu)(E) times the probability 1 - exp(-mu_i(E) x_i) that the photon
interacts along its path; the mean over the N_i rays divided by the phantom
mass M is D_0(E) (Eq. 6), and the fluence-weighted sum over energies is the
dose per particle D_p (Eq. 7).  Readings taken here:

* mu_i(E) x_i is the ray's projection at energy E, sum_m mu[m][E] L_i,m (for
  the paper's water phantom this is mu_water(E) x_i);
* mu_en / mu is one table per energy (water's, as in the paper), given in;
* the rays are every detector pixel of the listed angles, hit or not
  (N_i counts them all), so D_0 is the mean over the listed projections;
* E, M and phi come in whatever units the caller uses; D_0 is then in units
  of E / M per particle, and phi is used as given (normalise it to 1 for a
  dose per particle of the spectrum).
"""
from __future__ import annotations

import numpy as np


def dose_per_particle(L, mu, energies, mu_en_over_mu, phi, mass, n_rays=None):
    """D_0[E] (Eq. 6) and D_p (Eq. 7) from path lengths L [..., M] of the rays.

    mu [M][E]; energies, mu_en_over_mu, phi [E]; mass > 0.  n_rays (N_i)
    defaults to the number of rays in L; a larger value stands for rays left
    out of L because they miss the phantom (L = 0 adds exactly 0).
    """
    L = np.asarray(L, np.float64)
    n_mat = L.shape[-1]
    L2 = L.reshape(-1, n_mat)
    n_rays = L2.shape[0] if n_rays is None else int(n_rays)
    mu = np.asarray(mu, np.float64)
    S = np.zeros(mu.shape[1])
    for r0 in range(0, L2.shape[0], 1 << 16):     # blocks of rays, to bound memory
        P = L2[r0:r0 + (1 << 16)] @ mu            # [rays][E]: projection per ray and energy
        S += (-np.expm1(-P)).sum(axis=0)          # 1 - exp(-P)
    per_photon = np.asarray(energies, np.float64) * np.asarray(mu_en_over_mu, np.float64)
    D0 = per_photon * S / (n_rays * float(mass))
    Dp = float((np.asarray(phi, np.float64) * D0).sum())
    return D0, Dp
