"""Oracle of the refinement driver: the rounds of unconstrained label
propagation (Section 6) followed by the rounds of unconstrained FM with the
penalty schedule and the switch to constrained rounds (Section 5.5), written
out plainly over the oracle's round. Test infrastructure only.

Readings (stated where the paper leaves room):
* A label-propagation round is the deterministic round with no penalty
  (mode 2) restricted to the active nodes, followed by rebalancing (which the
  round does whenever a block is overloaded). Its net improvement is the cut
  before minus the cut after. If it is not positive, the partition is rolled
  back to the round's start and the phase ends. Otherwise the next active set
  is every node that did not move and has a neighbour that moved. The phase
  starts from the boundary nodes and ends after `lp_rounds` rounds, on an empty
  active set, or when the improvement falls below lp_min_rel times the cut
  before the round.
* The FM phase runs at most `fm_rounds` rounds. While unconstrained, round i
  is penalised with tau_i (linear from tau_1 to 1 over the unconstrained
  rounds, fm_rounds - 1 of them at most) and the phase switches to constrained
  rounds once a round improves the cut by less than fm_switch_rel times its
  starting cut. Constrained rounds then run until one improves by less than
  that threshold or the budget ends; at least one constrained round runs (the
  last round of the budget is always constrained).
"""
from fractions import Fraction

import numpy as np

from oracle import oracle as O


def boundary(g, part):
    """Nodes with a neighbour in another block."""
    out = np.zeros(g.n, np.uint8)
    for v in range(g.n):
        for e in range(g.xadj[v], g.xadj[v + 1]):
            if part[g.adjncy[e]] != part[v]:
                out[v] = 1
                break
    return out


def next_active(g, before, after):
    """Nodes that did not move and have a neighbour that moved."""
    moved = before != after
    out = np.zeros(g.n, np.uint8)
    for v in range(g.n):
        if moved[v]:
            continue
        for e in range(g.xadj[v], g.xadj[v + 1]):
            if moved[g.adjncy[e]]:
                out[v] = 1
                break
    return out


def tau_linear(i, rounds, tau1):
    """tau_1 + (1 - tau_1) (i - 1) / (rounds - 1) as a rational (num, den)."""
    t1 = Fraction(*tau1)
    t = t1 if rounds <= 1 else t1 + (1 - t1) * Fraction(i - 1, rounds - 1)
    return (t.numerator, t.denominator)


def refine(g, k, part, eps=(3, 100), lp_rounds=5, lp_min_rel=(1, 1000), fm_rounds=10,
           tau1=(1, 2), fm_switch_rel=(2, 1000), seq_penalty=1):
    """Run the driver in place on `part`. Returns the list of per-round
    records (phase, kind, stats) in order; phase 'lp' or 'fm', kind the mode
    ('lp', 'unconstrained', 'constrained', 'rollback')."""
    G = O.Graph(g)
    conn = np.zeros(max(g.n * k, 1), np.int32)
    W = np.zeros(k, np.int64)
    log = []
    # label propagation
    active = boundary(g, part)
    for _ in range(lp_rounds):
        if not active.any():
            break
        start = part.copy()
        st, _ = O.refine_round(G, O.params(k, eps, mode=2, seq_penalty=seq_penalty), part, conn, W,
                               active=active)
        before, after = int(st[1]), int(st[3])
        log.append(("lp", "lp", st.copy()))
        if after >= before:
            part[:] = start
            log.append(("lp", "rollback", st.copy()))
            break
        active = next_active(g, start, part)
        if Fraction(before - after) < Fraction(*lp_min_rel) * before:
            break
    # FM with the penalty schedule and the switch to constrained rounds
    unconstrained = True
    n_unc = max(fm_rounds - 1, 1)
    done = 0
    i = 0
    while done < fm_rounds:
        last = done == fm_rounds - 1
        if unconstrained and not last:
            i += 1
            p = O.params(k, eps, tau=tau_linear(i, n_unc, tau1), mode=0, seq_penalty=seq_penalty)
            kind = "unconstrained"
        else:
            unconstrained = False
            p = O.params(k, eps, mode=1, seq_penalty=seq_penalty)
            kind = "constrained"
        st, _ = O.refine_round(G, p, part, conn, W)
        done += 1
        log.append(("fm", kind, st.copy()))
        before, after = int(st[1]), int(st[3])
        small = Fraction(before - after) < Fraction(*fm_switch_rel) * max(before, 1)
        if kind == "unconstrained" and small:
            unconstrained = False
        elif kind == "constrained" and small:
            break
    return log
