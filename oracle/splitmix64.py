"""SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): a 64-bit counter advanced by the golden-ratio
increment, passed through a fixed 64-bit finalizer.

The k-means++ seeding draws (the paper's K-means++ subsection: the first
prototype uniformly at random, the next ones with probability proportional
to the squared distance) use this stream: the first draw picks the first
centre as ``next() % F``, each later draw is ``next() % T`` with T the exact
integer sum of squared distances (binary data), or ``(next() >> 11) * 2^-53``
scaled by T for real-valued data.
"""

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB


class SplitMix64:
    def __init__(self, seed: int):
        self.state = int(seed) & MASK64

    def next(self) -> int:
        self.state = (self.state + GOLDEN_GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * MIX1) & MASK64
        z = ((z ^ (z >> 27)) * MIX2) & MASK64
        return z ^ (z >> 31)

    def next_unit(self) -> float:
        """A double in [0, 1) from the top 53 bits of the next draw."""
        return (self.next() >> 11) * (1.0 / (1 << 53))
