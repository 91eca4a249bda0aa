"""The paper's I/O model and a red-blue pebble simulator.  TEST INFRASTRUCTURE ONLY.

Independent of the product planner; the tests compare the two and pin this
module to the numbers the paper prints.  S is the fast-memory size in
words, one word per matrix element (section 2.1, section 2.4).

Readings of the paper taken here (each is restated where it is used):
  * eq. aopt / eq. bopt use floors that are not the integer optimum of the
    problem they solve; ``seq_tile_search`` solves that problem exactly and
    ``seq_tile_closed`` evaluates the printed closed forms.
  * Theorem 2's min{} is a valid but loose bound; the schedule's own cost is
    ``par_schedule_cost`` = 2mnk/(p a) + a^2 with a from eq. optTileShape.
  * Grid fitting (section 7.1) gives no formula: over p' in
    [ceil((1-delta) p), p] and every factorisation p' = pm*pn*pk, minimise
    the local-domain surface (m/pm)(k/pk) + (n/pn)(k/pk) + (m/pm)(n/pn);
    ties go to the larger p'.
"""
from __future__ import annotations

import math


# ---------------------------------------------------------------- section 5
def thm1_bound(m: int, n: int, k: int, S: float) -> float:
    """Theorem 1: any pebbling needs at least 2mnk/sqrt(S) + mn I/O operations."""
    return 2.0 * m * n * k / math.sqrt(S) + m * n


def xs_schedule_io(m: int, n: int, k: int, S: float) -> float:
    """I/O of the X = S greedy schedule of section 5 (outer products of
    vectors of length sqrt(S+1) - 1): 2mnk/(sqrt(S+1)-1) + mn."""
    return 2.0 * m * n * k / (math.sqrt(S + 1.0) - 1.0) + m * n


def xs_factor(S: float) -> float:
    """Ratio of the X = S schedule to the lower bound, sqrt(S)/(sqrt(S+1)-1)
    (section 5, Corollary)."""
    return math.sqrt(S) / (math.sqrt(S + 1.0) - 1.0)


def rho_seq(a: int, b: int) -> float:
    """Computational intensity ab/(a+b) of one outer-product step (section 5)."""
    return a * b / (a + b)


def seq_tile_closed(S: int):
    """eq. aopt and eq. bopt as printed (floors of the closed forms)."""
    r = math.sqrt((S - 1.0) ** 3)
    a = math.floor((r - S + 1.0) / (S - 2.0))
    b = math.floor(-(2.0 * S + r - S * S - 1.0) / (r - S + 1.0))
    return a, b


def seq_tile_search(S: int):
    """Integer optimum of: maximise ab/(a+b) s.t. ab + a + 1 <= S, a,b >= 1
    (section 5).  Ties keep the smaller a.  Returns (a, b, rho)."""
    best = (0, 0, -1.0)
    for a in range(1, S):
        b = (S - 1 - a) // a
        if b < 1:
            break
        rho = rho_seq(a, b)
        if rho > best[2] + 1e-15 * rho:
            best = (a, b, rho)
    return best


def seq_greedy_io(m: int, n: int, k: int, a: int, b: int) -> float:
    """I/O of the greedy schedule with an a x b block of C resident (section 5,
    Corollary): mnk (a+b)/(ab) loads plus mn stores."""
    return m * n * k * (a + b) / (a * b) + m * n


# ---------------------------------------------------------------- section 6
def p1(m: int, n: int, S: float) -> float:
    """Number of dependency-free sqrt(S) x sqrt(S) x k domains, mn/S (section 6.2)."""
    return m * n / S


def ij_per_proc_io(m: int, n: int, k: int, p: int, S: float) -> float:
    """Per-processor I/O for p <= p1 (section 6.2): 2mnk/(p sqrt(S)) + mn/p."""
    return 2.0 * m * n * k / (p * math.sqrt(S)) + m * n / p


def opt_tile_shape(m: int, n: int, k: int, p: int, S: float):
    """eq. optTileShape: a = min{sqrt S, (mnk/p)^(1/3)}, b = max{mnk/(pS), (mnk/p)^(1/3)}."""
    c = (m * n * k / p) ** (1.0 / 3.0)
    return min(math.sqrt(S), c), max(m * n * k / (p * S), c)


def thm2_bound(m: int, n: int, k: int, p: int, S: float) -> float:
    """Theorem 2 as printed: min{2mnk/(p sqrt S) + S, 3 (mnk/p)^(2/3)}."""
    return min(2.0 * m * n * k / (p * math.sqrt(S)) + S, 3.0 * (m * n * k / p) ** (2.0 / 3.0))


def par_schedule_cost(m: int, n: int, k: int, p: int, S: float) -> float:
    """Per-processor I/O of the schedule itself, Q = 2mnk/(p a) + a^2 with a
    from eq. optTileShape (I/O-latency trade-off, section 6.3)."""
    a, _ = opt_tile_shape(m, n, k, p, S)
    return 2.0 * m * n * k / (p * a) + a * a


def latency_rounds(a: float, b: float, S: float) -> int:
    """L = ceil(2ab / (S - a^2)) communication rounds (section 6.3)."""
    return math.ceil(2.0 * a * b / (S - a * a))


def step_size(S: int, a: int) -> int:
    """Algorithm 1 step size s = floor((S - a^2) / (2a)) outer products per round."""
    return (S - a * a) // (2 * a)


# ---------------------------------------------------------------- section 7.1
def grid_surface(m: int, n: int, k: int, g) -> float:
    pm, pn, pk = g
    return (m / pm) * (k / pk) + (n / pn) * (k / pk) + (m / pm) * (n / pn)


def _factor_triples(q: int):
    for pm in range(1, q + 1):
        if q % pm:
            continue
        r = q // pm
        for pn in range(1, r + 1):
            if r % pn:
                continue
            yield pm, pn, r // pn


def fit_ranks(m: int, n: int, k: int, p: int, delta: float):
    """Grid fitting with at most a fraction delta of idle processors (section 7.1).

    Returns (grid, used) minimising the local-domain surface; ties go to the
    larger number of used processors."""
    lo = max(1, math.ceil((1.0 - delta) * p - 1e-9))
    best = None
    for q in range(p, lo - 1, -1):
        for g in _factor_triples(q):
            s = grid_surface(m, n, k, g)
            if best is None or s < best[0] * (1 - 1e-12):
                best = (s, g, q)
    return best[1], best[2]


# ---------------------------------------------------------------- pebbling
class PebbleError(AssertionError):
    pass


def simulate_tiled(m: int, n: int, k: int, tile_m: int, tile_n: int, kc: int, p_k: int,
                   S: int, beta_nonzero: bool = False):
    """Play the red-blue pebble game (section 2.2) for the tiled schedule.

    Work item = (row block, column block, k split).  For each item the partial
    sums of its tile_m x tile_n block of C hold red pebbles for the whole item
    (an accumulator is updated in place: the pebble of C(i,j,t) slides to
    C(i,j,t+1)); the reduction range of the split is walked in rounds of kc,
    each round loading a tile_m x kc block of A and a kc x tile_n block of B,
    then computing every update of the round and freeing the round's inputs.
    With p_k == 1 the final block is stored (plus C0 loads if beta != 0).
    With p_k > 1 each item stores its partial block; the reduction then, per
    entry, loads the p_k partials (and C0), computes and stores the result.

    The number of red pebbles is checked against S after every move.  Returns
    the I/O count (loads + stores) in words.
    """
    red = set()
    io = 0

    def place(v):
        red.add(v)
        if len(red) > S:
            raise PebbleError(f"{len(red)} red pebbles > S = {S}")

    ksplit = [(k * s) // p_k for s in range(p_k + 1)]
    for i0 in range(0, m, tile_m):
        for j0 in range(0, n, tile_n):
            rows = range(i0, min(i0 + tile_m, m))
            cols = range(j0, min(j0 + tile_n, n))
            for s in range(p_k):
                kb, ke = ksplit[s], ksplit[s + 1]
                acc = {}
                for r0 in range(kb, ke, kc):
                    rr = range(r0, min(r0 + kc, ke))
                    for i in rows:
                        for t in rr:
                            place(("a", i, t)); io += 1
                    for t in rr:
                        for j in cols:
                            place(("b", t, j)); io += 1
                    for t in rr:
                        for i in rows:
                            for j in cols:
                                if ("a", i, t) not in red or ("b", t, j) not in red:
                                    raise PebbleError("operand not red")
                                prev = acc.get((i, j))
                                if prev is not None:
                                    red.discard(prev)
                                v = ("c", s, i, j, t)
                                place(v)
                                acc[(i, j)] = v
                    for i in rows:
                        for t in rr:
                            red.discard(("a", i, t))
                    for t in rr:
                        for j in cols:
                            red.discard(("b", t, j))
                if p_k == 1:
                    for i in rows:
                        for j in cols:
                            if beta_nonzero:
                                place(("c0", i, j)); io += 1
                                red.discard(("c0", i, j))
                            io += 1  # store the final entry
                            red.discard(acc.get((i, j)))
                else:
                    for i in rows:
                        for j in cols:
                            io += 1  # store the partial entry
                            red.discard(acc.get((i, j)))
    if p_k > 1:
        for i in range(m):
            for j in range(n):
                for s in range(p_k):
                    place(("p", s, i, j)); io += 1
                if beta_nonzero:
                    place(("c0", i, j)); io += 1
                for s in range(p_k):
                    red.discard(("p", s, i, j))
                red.discard(("c0", i, j))
                io += 1  # store C
    return io
