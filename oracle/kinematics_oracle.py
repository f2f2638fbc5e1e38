"""Pair kinematics of colliding photon pairs (Sec. 1, Eqs. pTotal and Lorentz): the
electron and positron each photon pair creates, in the lab frame.

TEST INFRASTRUCTURE ONLY: the product library never imports this module; only the tests,
the smoke check and the benchmark's CPU baseline do. It shares no code with the GPU path.

Steps, in the paper's order (units MeV, c = 1, m_e = 0.51099895 MeV):
  1. E_tot = E_i + E_j, p_tot = p_i + p_j (lab frame);
  2. centre-of-mass momentum of each lepton, p' = sqrt([E_tot^2 - p_tot^2] / 4 - m_e^2)
     (the printed equation subtracts m_e c^2 under the root; the dimensions require
     m_e^2 c^4, i.e. m_e^2 with c = 1); the lepton's CoM energy is sqrt(p'^2 + m_e^2);
  3. the direction of the positron in the CoM frame is random and isotropic (the paper
     draws it at random); the electron moves in the exact opposite direction. The draw is
     reproducible: cos(theta) = 2 u0 - 1 and phi = 2 pi u1, u0 and u1 the top 53 bits of
     the first two 64-bit words of Philox4x64-10 (Salmon et al., "Parallel random numbers:
     as easy as 1, 2, 3", SC'11) at counter (k, i, j, 0) and key (seed, 0), times 2^-53;
  4. CoM velocity beta_CoM = p_tot / E_tot; each lepton's CoM velocity beta' (magnitude
     p' / E', along its direction) is carried to the lab by relativistic velocity
     addition: beta = (beta_CoM + beta'_par + beta'_perp sqrt(1 - beta_CoM^2)) /
     (1 + beta' . beta_CoM), beta'_par the part of beta' along beta_CoM and beta'_perp =
     beta' - beta'_par (the printed equation writes an unprimed beta_perp and defines it
     as beta_CoM - beta'_par; the velocity-addition law needs the component of beta'
     perpendicular to beta_CoM);
  5. lab Lorentz factor gamma = 1 / sqrt(1 - beta^2), energy gamma m_e, momentum
     gamma m_e beta.
Histograms: the positron's Lorentz factor (caller edges) and its polar angle to +z over
[0, pi] (n equal bins), each hit weighted by sqrt(w_i w_j), the photons it represents.
"""
import math

import numpy as np

ME = 0.51099895
_MASK = (1 << 64) - 1
_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B


def philox4x64(counter, key):
    """Philox4x64-10 block: ten rounds of two 64x64 -> 128-bit products with the
    published multipliers, the key bumped by the published Weyl constants between rounds."""
    x = [int(v) & _MASK for v in counter]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * x[0]
        p1 = _M1 * x[2]
        x = [(p1 >> 64) ^ x[1] ^ k0, p1 & _MASK, (p0 >> 64) ^ x[3] ^ k1, p0 & _MASK]
    return x


def uniforms(seed, k, i, j):
    """The two uniform numbers in [0, 1) of hit (k, i, j)."""
    r = philox4x64((k, i, j, 0), (seed, 0))
    return (r[0] >> 11) * 2.0 ** -53, (r[1] >> 11) * 2.0 ** -53


def cm_direction(seed, k, i, j):
    u0, u1 = uniforms(seed, k, i, j)
    ct = 2.0 * u0 - 1.0
    st = math.sqrt(max(0.0, 1.0 - ct * ct))
    phi = 2.0 * math.pi * u1
    return (st * math.cos(phi), st * math.sin(phi), ct)


def _lab_velocity(bc, bp):
    """Velocity addition of CoM velocity bc and CoM-frame velocity bp (step 4)."""
    b2 = (bc[0] * bc[0] + bc[1] * bc[1]) + bc[2] * bc[2]
    dot = (bp[0] * bc[0] + bp[1] * bc[1]) + bp[2] * bc[2]
    if not (b2 > 0.0):
        return bp
    f = dot / b2
    par = (f * bc[0], f * bc[1], f * bc[2])
    perp = (bp[0] - par[0], bp[1] - par[1], bp[2] - par[2])
    root = math.sqrt(1.0 - b2)
    den = 1.0 + dot
    return tuple((bc[a] + par[a] + perp[a] * root) / den for a in range(3))


def pair_leptons(Ei, pi, Ej, pj, seed, k, i, j):
    """(positron E, px, py, pz), (electron E, px, py, pz), CoM direction of the positron."""
    Et = Ei + Ej
    pt = (pi[0] + pj[0], pi[1] + pj[1], pi[2] + pj[2])
    p2 = (pt[0] * pt[0] + pt[1] * pt[1]) + pt[2] * pt[2]
    pcm = math.sqrt(max(0.0, (Et * Et - p2) / 4.0 - ME * ME))
    ecm = math.sqrt(pcm * pcm + ME * ME)
    n = cm_direction(seed, k, i, j)
    bmag = pcm / ecm
    bc = (pt[0] / Et, pt[1] / Et, pt[2] / Et)
    out = []
    for sgn in (1.0, -1.0):
        bp = (sgn * bmag * n[0], sgn * bmag * n[1], sgn * bmag * n[2])
        b = _lab_velocity(bc, bp)
        bb = (b[0] * b[0] + b[1] * b[1]) + b[2] * b[2]
        g = 1.0 / math.sqrt(1.0 - bb)
        out.append((g * ME, g * ME * b[0], g * ME * b[1], g * ME * b[2]))
    return out[0], out[1], n


def kinematics(A, B, i, j, k, seed):
    """Leptons of every pair (rows i of beam A, rows j of beam B, steps k): arrays of shape
    (n, 4) for the positrons and the electrons."""
    pos = np.zeros((len(i), 4))
    ele = np.zeros((len(i), 4))
    for h in range(len(i)):
        a, b, s = int(i[h]), int(j[h]), int(k[h])
        p, e, _ = pair_leptons(A["E"][a], (A["px"][a], A["py"][a], A["pz"][a]),
                               B["E"][b], (B["px"][b], B["py"][b], B["pz"][b]), seed, s, a, b)
        pos[h] = p
        ele[h] = e
    return pos, ele


def histograms(A, B, i, j, pos, gamma_edges, n_theta):
    """Positron Lorentz-factor and polar-angle histograms weighted by sqrt(w_i w_j)."""
    w = np.sqrt(A["w"][i] * B["w"][j])
    g = pos[:, 0] / ME
    gh = np.zeros(len(gamma_edges) - 1)
    b = np.searchsorted(gamma_edges, g, side="right") - 1
    ok = (b >= 0) & (b < len(gamma_edges) - 1)
    np.add.at(gh, b[ok], w[ok])
    th = np.array([math.atan2(math.hypot(px, py), pz) for px, py, pz in pos[:, 1:]])
    tb = np.minimum((th / math.pi * n_theta).astype(np.int64), n_theta - 1)
    thh = np.zeros(n_theta)
    np.add.at(thh, tb, w)
    return gh, thh
