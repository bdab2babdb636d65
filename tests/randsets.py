"""Seeded random token sets over small alphabets (input generation for the sweeps).

Each set has 1-4 kinds; each kind is a random regex of depth <= 3 over literals, classes,
concatenation, alternation and the postfix operators * + ?, with a random priority and a
random discard flag, as in the exhaustive validation of Section 6.1.
"""
import random


def rand_regex(rng: random.Random, alphabet: str, depth: int) -> str:
    if depth == 0 or rng.random() < 0.3:
        r = rng.random()
        if r < 0.6:
            return rng.choice(alphabet)
        k = rng.randint(1, len(alphabet))
        chars = "".join(sorted(rng.sample(alphabet, k)))
        return "[" + chars + "]"
    r = rng.random()
    if r < 0.35:
        n = rng.randint(2, 3)
        return "".join(_group(rand_regex(rng, alphabet, depth - 1)) for _ in range(n))
    if r < 0.6:
        n = rng.randint(2, 3)
        return "(" + "|".join(rand_regex(rng, alphabet, depth - 1) for _ in range(n)) + ")"
    op = rng.choice("*+?")
    return _group(rand_regex(rng, alphabet, depth - 1)) + op


def _group(s: str) -> str:
    if len(s) == 1 or (s.startswith("[") and s.endswith("]") and s.count("[") == 1):
        return s
    if s.startswith("(") and s.endswith(")") and _balanced_inner(s):
        return s
    return "(" + s + ")"


def _balanced_inner(s: str) -> bool:
    d = 0
    for i, c in enumerate(s):
        d += c == "("
        d -= c == ")"
        if d == 0 and i < len(s) - 1:
            return False
    return True


def rand_set(seed: int, alphabet: str = "abc"):
    rng = random.Random(seed)
    k = rng.randint(1, 4)
    return [(rand_regex(rng, alphabet, 3), rng.randint(0, 2), rng.random() < 0.4) for _ in range(k)]
