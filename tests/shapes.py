"""Hand-built tree shapes for planner and parity tests (inputs only)."""
import numpy as np

from paper_1202_3777_amd.instances import from_arrays


def hub_with_chains(seed: int = 0, n_slots: int = 4):
    """A hub clique of 6 variables with 14 chains hanging from it, of 1..7
    cliques each (two of every length), so the hub is the tree's center and,
    in the schedule's orientation, has 14 children that finish at heights
    0..6.  Each chain clique shares 2 variables with its parent and adds 2
    fresh ones; cardinalities 2 and 3.  Evidence: slot 0 none, slot 1 at the
    end of a longest chain, slot 2 on a hub variable, slot 3 in three chains.
    Returns the instance and the hub's index (0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    card = []

    def new_var():
        card.append(int(rng.integers(2, 4)))
        return len(card) - 1

    hub = [new_var() for _ in range(6)]
    cliques, parent = [hub], [-1]
    ends = []
    for i in range(14):
        length = i % 7 + 1
        prev, prev_vars = 0, hub
        for _ in range(length):
            shared = list(rng.choice(prev_vars, size=2, replace=False))
            vars_ = shared + [new_var(), new_var()]
            rng.shuffle(vars_)
            cliques.append([int(v) for v in vars_])
            parent.append(prev)
            prev, prev_vars = len(cliques) - 1, cliques[-1]
        ends.append(prev)
    fresh = lambda c: [v for v in cliques[c] if v not in cliques[parent[c]]]   # noqa: E731
    longest = ends[6]
    evidence = [([], []),
                ([fresh(longest)[0]], [1]),
                ([hub[2]], [0]),
                ([fresh(ends[1])[0], fresh(ends[9])[1], fresh(ends[12])[0]], [0, 1, 1])]
    evidence = [(np.asarray(v, np.int32), np.asarray(s, np.int32)) for v, s in evidence[:n_slots]]
    inst = from_arrays(card, cliques, parent, evidence=evidence, seed=seed, name="hub-with-chains")
    return inst, 0


def paired_tiles(seed: int = 0):
    """A clique of 10 variables (cardinality 3 eight times, then 2, 2: its tile
    is the last five variables, 108 entries, and it has 243 tiles) with 6
    children of 4 variables each (2 shared, 2 fresh), and a grandchild under
    the first child.  Tiles of at most 128 entries are streamed two to a
    wave, and an odd tile count leaves a half-wave idle on the last step;
    two of the children's separators are reduced in wave groups, the other
    four in block groups.
    Six evidence sets: none, an outer variable of the big clique (whole
    tiles zeroed), an inner one (masked positions), both, child variables,
    and the same as the first to share a multi-slot set."""
    rng = np.random.Generator(np.random.PCG64(seed))
    card = [3, 3, 3, 3, 3, 3, 3, 3, 2, 2]
    big = list(range(10))
    cliques, parent = [big], [-1]
    shared = [(0, 5), (1, 7), (2, 3), (4, 9), (0, 6), (3, 1)]
    for a, b in shared:
        f0, f1 = len(card), len(card) + 1
        card += [int(rng.integers(2, 4)), int(rng.integers(2, 4))]
        cliques.append([a, f0, b, f1])
        parent.append(0)
    g0 = len(card)
    card += [2, 3]
    cliques.append([cliques[1][1], g0, cliques[1][3], g0 + 1])
    parent.append(1)
    evidence = [([], []), ([1], [2]), ([6], [0]), ([0, 7], [1, 1]),
                ([cliques[3][1], g0 + 1], [1, 2]), ([], [])]
    inst = from_arrays(card, cliques, parent, evidence=evidence, seed=seed, name="paired-tiles")
    return inst
