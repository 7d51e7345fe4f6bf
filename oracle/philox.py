"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from the
published definition.  Oracle-only implementation.

The paper's optical-depth method (App. B) draws uniform numbers x_r in (0,1)
without fixing a generator.  Both the oracle and the HIP path use this
counter-based stream so a particle's draws depend only on
(particle id, run seed, step, slot) and not on thread or processing order:
  key     = (id, seed)
  counter = (step, slot, 0, 0)
A 32-bit output x maps to u = ((x >> 9) + 0.5) * 2^-23, which lies strictly
inside (0, 1) and is exactly representable in both FP32 and FP64.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: 4 arrays (or scalars) of uint32 values, key: 2.  Returns 4 uint64
    arrays holding the 32-bit outputs.  Ten rounds, key bumped between
    rounds by the Weyl constants."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & _MASK for v in ctr)
    k0, k1 = (np.asarray(v, dtype=np.uint64) & _MASK for v in key)
    for rnd in range(10):
        p0 = _M0 * c0                       # 32x32 -> 64-bit products
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
        if rnd < 9:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def to_uniform(x):
    """32-bit integer -> double in (0, 1), 23 significant bits."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def uniforms(ids, seed, step, slot):
    """Four uniforms per particle for (step, slot)."""
    ids = np.asarray(ids, dtype=np.uint64)
    z = np.zeros_like(ids)
    out = philox4x32_10((z + np.uint64(step), z + np.uint64(slot), z, z),
                        (ids, z + np.uint64(seed)))
    return tuple(to_uniform(o) for o in out)


# Slot numbers of the per-step draws: Davies scatter and photon energy,
# photon angles and new optical depth, reflux on x / y / z, injection.
SLOT_COLLIDE = 0
SLOT_PHOTON = 1
SLOT_REFLUX = (2, 3, 4)
SLOT_INJECT_A = 8
SLOT_INJECT_B = 9
# Delta rays: azimuth and new optical depth of an emission; optical depths
# of a newborn delta ray (keyed by its own id); rejection candidates of the
# energy sampler, two per slot, in slots SLOT_DELTA_TRY .. SLOT_DELTA_TRY + 15.
SLOT_DELTA_K = 12
SLOT_BIRTH = 13
SLOT_DELTA_TRY = 16
