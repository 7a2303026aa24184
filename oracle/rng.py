"""Counter-based random numbers for the genetic algorithm (oracle side).

Every random number the search draws is a pure function of its coordinates
(seed, run, generation, individual, purpose, index), so an independent
implementation that follows the same definition draws the same numbers in any
order.  The mixing function is SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): add the golden-ratio
increment, then two xor-shift-multiply rounds and a final xor-shift.

A draw folds each coordinate into the state in turn, h <- splitmix64(h xor c),
starting from h = seed, and keeps the top 24 bits.  A 24-bit integer u is exactly
representable in float32, so u / 2^24 is the same number in FP32 and FP64.
"""
M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB

# purposes (which decision a draw feeds)
P_INIT = 1
P_TOURNAMENT = 2
P_CROSSOVER = 3
P_MUTATION = 4
P_LS_PICK = 5
P_LS_SW = 6


def splitmix64(x: int) -> int:
    z = (x + GOLDEN) & M64
    z = ((z ^ (z >> 30)) * MIX1) & M64
    z = ((z ^ (z >> 27)) * MIX2) & M64
    return z ^ (z >> 31)


def draw_u24(seed: int, run: int, gen: int, indiv: int, purpose: int, index: int) -> int:
    h = seed & M64
    for c in (run, gen, indiv, purpose, index):
        h = splitmix64(h ^ (c & M64))
    return h >> 40


def uniform(seed, run, gen, indiv, purpose, index) -> float:
    """Uniform in [0, 1) with 24-bit resolution."""
    return draw_u24(seed, run, gen, indiv, purpose, index) / 16777216.0


def randint(n: int, seed, run, gen, indiv, purpose, index) -> int:
    """Integer uniform in [0, n): (u24 * n) >> 24, exact in integer arithmetic."""
    return (draw_u24(seed, run, gen, indiv, purpose, index) * n) >> 24
