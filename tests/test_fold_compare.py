"""The bit-packed kernels' folded compare, modelled word by word on the CPU.

A bit-packed site draws its uniform u as 32 bit-sliced levels (level k = bit
31 - k of u, one RNG word per level for 32 sites) and becomes +1 iff u < T,
T the threshold of its class (the threshold contract: T from the field h in
double, T(h) + T(-h) = 2^32).  The kernels compare in a flipped domain: with
mirror classes of equal t and opposite signs (a class with T = 2^31 may take
either sign), the flip plane is smask = c ^ F(class) and the class words are
tf = t ^ F, so each site compares u with y = tf ^ c; the new spin is y's bit at
the most significant level where u and y differ, smask where all 32 agree.
Levels 0..7 run least significant first, deeper levels most significant first.

This model restates that design with plain integer bit operations and checks
it against u < T site by site, for the square lattice (three folded classes)
and the triangular lattice (four agreement classes), on random words and on
words forced to tie with y down to every depth, with tables where classes have
h = 0, J < 0, beta = 0 and lambda = 0.  The thresholds come from the oracle.
It checks the design, not the kernels: those are checked against the oracle by
the GPU parity tests.
"""
import random

import pytest

import oracle

M32 = 0xFFFFFFFF


def ones(word, sh):
    return M32 if (word >> sh) & 1 else 0


def tables(J, q, lam, beta, nb):
    """Class thresholds, t words and flip bits of the folded table (classes
    j = n_plus + (nb + 1) c), and whether the table folds."""
    ncl = 2 * (nb + 1)
    T, t, sgn = [], [], 0
    for j in range(ncl):
        nplus, cb = j % (nb + 1), j // (nb + 1)
        h = oracle.field(J * (2 * nplus - nb), 1 if cb else -1, q, lam)
        Tj = oracle.threshold(h, beta)
        T.append(Tj)
        t.append(((1 << 32) - Tj if h >= 0 else Tj) & M32)
        if h >= 0:
            sgn |= 1 << j
    fold = True
    for j in range(ncl // 2):
        k = ncl - 1 - j
        fold = fold and t[j] == t[k]
        if ((sgn >> j) ^ (sgn >> k)) & 1:
            continue
        if T[k] == 1 << 31:
            sgn ^= 1 << k
        elif T[j] == 1 << 31:
            sgn ^= 1 << j
        else:
            fold = False
    return T, t, sgn, fold


def square_classes(a, b, c):
    """(plane, class word index, flip bit index) of the three folded classes."""
    one = a ^ b
    al = ~(a ^ c) & ~one & M32
    rest = ~one & ~al & M32
    return [(one, 1, 1), (al, 0, 0), (rest, 2, 2)]


def tri_classes(a, b, e, c):
    """The four agreement classes k: class word t_{4+k}, flip bit 3 - k."""
    xa, xb, xe = ~(a ^ c) & M32, ~(b ^ c) & M32, ~(e ^ c) & M32
    s1 = xa ^ xb ^ xe
    s2 = (xa & xb) | (xa & xe) | (xb & xe)
    planes = [~s1 & ~s2 & M32, s1 & ~s2, ~s1 & s2, s1 & s2]
    return [(planes[k], 4 + k, 3 - k) for k in range(4)]


def folded_word(classes, c, vm, R, t, sgn):
    def tf_bit(k):
        out = 0
        for plane, ti, fi in classes:
            out |= plane & ones(t[ti] ^ ones(sgn, fi), 31 - k)
        return out

    o, eq = 0, M32
    for k in range(7, -1, -1):          # least significant first
        y = tf_bit(k) ^ c
        diff = R[k] ^ y
        o = (diff & y) | (~diff & o & M32)
        eq &= ~diff & M32
    und, out = eq & vm, o & ~eq & M32
    for k in range(8, 32):              # most significant first
        if und == 0:
            break
        d = R[k] ^ c ^ tf_bit(k)
        e = und & d
        out |= e & ~R[k] & M32
        und &= ~d & M32
    if und:
        smask = c
        for plane, _, fi in classes:
            smask ^= plane & ones(sgn, fi)
        out |= und & smask
    return out & vm


def site_by_site(nplus_of, c, vm, R, T, nb):
    out = 0
    for i in range(32):
        if not (vm >> i) & 1:
            continue
        u = 0
        for k in range(32):
            u = (u << 1) | ((R[k] >> i) & 1)
        j = nplus_of(i) + (nb + 1) * ((c >> i) & 1)
        if u < T[j]:
            out |= 1 << i
    return out


CASES = [  # J, q, lambda, beta
    (1, 1.0, 0.0, 0.4),
    (1, 2.0, 0.0, 0.44),   # square lattice: the rest classes have h = 0
    (1, 0.5, 0.0, 0.3),
    (1, 0.0, 0.0, 0.5),    # q = 0: the one-neighbour classes have h = 0
    (-1, 2.0, 0.0, 0.4),   # J < 0
    (1, 1.0, 0.0, 0.0),    # beta = 0: every T = 2^31
    (2, 4.0, 0.0, 0.3),
    (1, 3.0, 0.0, 0.7),    # triangular lattice: classes with h = 0
]


def forced_ties(rng, classes, c, t, sgn, depth):
    """RNG words equal to every site's y on the first `depth` levels."""
    R = [rng.getrandbits(32) for _ in range(32)]
    for k in range(depth):
        y = c
        for plane, ti, fi in classes:
            y ^= plane & ones(t[ti] ^ ones(sgn, fi), 31 - k)
        R[k] = y & M32
    return R


@pytest.mark.parametrize("lattice", ["square", "triangular"])
@pytest.mark.parametrize("J,q,lam,beta", CASES)
def test_folded_compare_equals_u_below_T(lattice, J, q, lam, beta):
    nb = 2 if lattice == "square" else 3
    T, t, sgn, fold = tables(J, q, lam, beta, nb)
    assert fold, "lambda = 0 tables fold"
    rng = random.Random(f"{lattice} {J} {q} {beta}")
    for it in range(60):
        a, b, e, c = (rng.getrandbits(32) for _ in range(4))
        vm = M32 if it % 3 else (1 << rng.randint(1, 31)) - 1
        if lattice == "square":
            classes = square_classes(a, b, c)
            nplus = lambda i: ((a >> i) & 1) + ((b >> i) & 1)
        else:
            classes = tri_classes(a, b, e, c)
            nplus = lambda i: ((a >> i) & 1) + ((b >> i) & 1) + ((e >> i) & 1)
        if it % 4 == 0:
            R = forced_ties(rng, classes, c, t, sgn, rng.choice([8, 9, 12, 20, 31, 32]))
        else:
            R = [rng.getrandbits(32) for _ in range(32)]
        assert folded_word(classes, c, vm, R, t, sgn) == site_by_site(nplus, c, vm, R, T, nb), it


def test_sign_choice_only_where_T_is_half():
    """The flip bits the folded table needs differ from the field's signs only
    on classes with T = 2^31, where both signs decide alike."""
    for nb in (2, 3):
        for J, q, lam, beta in CASES:
            T, t, sgn, fold = tables(J, q, lam, beta, nb)
            for j in range(2 * (nb + 1)):
                nplus, cb = j % (nb + 1), j // (nb + 1)
                h = oracle.field(J * (2 * nplus - nb), 1 if cb else -1, q, lam)
                if ((sgn >> j) & 1) != (h >= 0):
                    assert T[j] == 1 << 31


def test_unequal_mirror_signs_do_not_fold():
    # q = 0, lambda != 0, J = 0: every class has h = lambda, mirror classes
    # the same sign and the same t -- the six-class table handles it
    T, t, sgn, fold = tables(0, 0.0, 0.5, 0.4, 2)
    assert not fold
    # the folded compare would be wrong there: the flip plane is not c ^ F
    rng = random.Random(5)
    wrong = 0
    for _ in range(20):
        a, b, c = (rng.getrandbits(32) for _ in range(3))
        R = [rng.getrandbits(32) for _ in range(32)]
        nplus = lambda i: ((a >> i) & 1) + ((b >> i) & 1)
        wrong += folded_word(square_classes(a, b, c), c, M32, R, t, sgn) != site_by_site(nplus, c, M32, R, T, 2)
    assert wrong > 0
