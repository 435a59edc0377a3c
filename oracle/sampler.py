"""Landmark sampler of the oracle (test infrastructure only).

Interpolation MDS starts from a random sample of l of the n points
(Section 3.1, "Interpolation MDS": the first data subset is drawn at random).
The paper names no generator, so both implementations follow one published
recipe, written independently on each side:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014; constants of the public-domain reference code):
  state += 0x9E3779B97F4A7C15, then a xor-shift/multiply finaliser.
* Lemire's bounded draw in [0, k) ("Fast random integer generation in an
  interval", ACM TOMACS 2019): take the high word of the 128-bit product
  next() * k, rejecting when the low word falls below (2^64 - k) mod k.
* Partial Fisher-Yates over a virtual identity permutation: for
  i = 0..l-1 swap a[i] with a[i + bounded(n - i)]; the landmarks are
  a[0..l-1], reported in ascending order.

Plain Python integers; slow and obviously correct.
"""

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB


class SplitMix64:
    """SplitMix64 generator; ``next()`` returns the next 64-bit output."""

    def __init__(self, seed):
        self.state = int(seed) & MASK64

    def next(self):
        self.state = (self.state + GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * MIX1) & MASK64
        z = ((z ^ (z >> 27)) * MIX2) & MASK64
        return z ^ (z >> 31)


def bounded(gen, k):
    """Uniform integer in [0, k) by Lemire's multiply-and-reject method."""
    k = int(k)
    if k <= 0:
        raise ValueError("bounded() needs k >= 1")
    prod = gen.next() * k
    low = prod & MASK64
    if low < k:
        threshold = ((1 << 64) - k) % k
        while low < threshold:
            prod = gen.next() * k
            low = prod & MASK64
    return prod >> 64


def fisher_yates_prefix(n, l, draw):
    """First l entries of a partial Fisher-Yates shuffle of 0..n-1.

    ``draw(k)`` must return an integer in [0, k).  Slots never touched hold
    their own index, so only the swapped ones are stored.
    """
    moved = {}
    for i in range(l):
        j = i + draw(n - i)
        ai = moved.get(i, i)
        aj = moved.get(j, j)
        moved[i] = aj
        moved[j] = ai
    return [moved.get(i, i) for i in range(l)]


def sample_landmarks(n, l, seed):
    """l distinct indices of 0..n-1, uniform without replacement, ascending."""
    n = int(n)
    l = int(l)
    if not (1 <= l <= n):
        raise ValueError("need 1 <= l <= n")
    gen = SplitMix64(seed)
    picked = fisher_yates_prefix(n, l, lambda k: bounded(gen, k))
    return sorted(picked)
