"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written from that paper's definition.

State: four 32-bit counter words and two 32-bit key words.  One round
multiplies counter words 0 and 2 by the two Philox multipliers, and forms the
new counter from the high halves xor-ed with the other two counter words and
the round key, and the low halves.  The key is advanced by the two Weyl
constants between rounds.  Ten rounds.

Test infrastructure only (see the package docstring).
"""

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_M32 = 0xFFFFFFFF


def philox4x32(ctr, key, rounds=10):
    """Return the 4 output words for counter ctr (4 words) and key (2 words)."""
    x0, x1, x2, x3 = (int(v) & _M32 for v in ctr)
    k0, k1 = (int(v) & _M32 for v in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + PHILOX_W0) & _M32
            k1 = (k1 + PHILOX_W1) & _M32
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0, p1 & _M32,
                          (p0 >> 32) ^ x3 ^ k1, p0 & _M32)
    return (x0, x1, x2, x3)


def seed_key(seed):
    seed = int(seed)
    return (seed & _M32, (seed >> 32) & _M32)


# Stream domains of the draw contract (counter word 1, bits 24..31).
DOM_EVENT = 1
DOM_BUDGET = 2
DOM_INIT = 3
DOM_PLAIN = 4
DOM_COMPONENT = 5


def event_plane_words(seed, net_id, group, event, n_planes):
    """Bit-plane draws of one event for one 32-lane group: plane q is output
    (q mod 4) of the call with plane-quad q//4.  Bit l of plane q is bit q of
    the threshold of replica 32*group + l."""
    planes = []
    for quad in range((n_planes + 3) // 4):
        ctr = (event & _M32,
               (DOM_EVENT << 24) | (quad << 16) | ((event >> 32) & 0xFFFF),
               group & _M32, net_id & _M32)
        out = philox4x32(ctr, seed_key(seed))
        planes.extend(out)
    return planes[:n_planes]


def event_threshold(seed, net_id, replica, event, n_planes):
    """Per-replica uniform integer on [0, 2^n_planes) from the plane words."""
    words = event_plane_words(seed, net_id, replica >> 5, event, n_planes)
    lane = replica & 31
    n = 0
    for q, w in enumerate(words):
        n |= ((w >> lane) & 1) << q
    return n


def plain_threshold(seed, net_id, replica, event, n_bits):
    """Per-replica draw of the one-replica-per-thread comparator: low n_bits
    of output (event mod 4) of the call keyed by event // 4."""
    blk = event >> 2
    ctr = (blk & _M32, (DOM_PLAIN << 24) | ((blk >> 32) & 0xFFFF),
           replica & _M32, net_id & _M32)
    out = philox4x32(ctr, seed_key(seed))
    return out[event & 3] & ((1 << n_bits) - 1)


def budget_uniform(seed, net_id, replica, advance):
    """64-bit uniform for the event budget of one replica in one advance."""
    ctr = (advance & _M32, (DOM_BUDGET << 24) | ((advance >> 32) & 0xFFFF),
           replica & _M32, net_id & _M32)
    out = philox4x32(ctr, seed_key(seed))
    return out[0] | (out[1] << 32)


def init_words(seed, net_id, replica, chunk):
    """128 random bits for initial-state draws of one replica."""
    ctr = (chunk & _M32, DOM_INIT << 24, replica & _M32, net_id & _M32)
    return philox4x32(ctr, seed_key(seed))


DOM_SHARED = 6


def shared_threshold(seed, net_id, e, Z):
    """n shared by every replica at event e: uniform on [0, Z) by 32-bit
    multiply-shift with rejection (Lemire) on output 0 of the SHARED draw;
    counter (e low 32, 6 << 24 | attempt << 16 | e bits 32..47, 0, net_id);
    the 256th attempt is taken as it is."""
    thresh = (2 ** 32 - Z) % Z
    m = 0
    for attempt in range(256):
        out = philox4x32((e & 0xFFFFFFFF, (DOM_SHARED << 24) | (attempt << 16) | ((e >> 32) & 0xFFFF),
                          0, net_id), seed_key(seed))
        m = out[0] * Z
        if (m & 0xFFFFFFFF) >= thresh:
            break
    return m >> 32
