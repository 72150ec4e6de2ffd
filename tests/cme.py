"""Brute-force chemical master equation on tiny networks (test reference).

The law of X(t) is the CME (paper, Methods section).  For a network with few
reachable states the CME is a finite linear ODE dp/dt = p Q, solved here as
p(t) = p(0) expm(Q t).  Propensities follow the combinatorial definition of
mass-action kinetics: c_j times the number of distinct reactant combinations,
prod_i binom(x_i, r_ij).  This is an independent statement of the model, not
the simulation code.
"""
from math import comb

import numpy as np
from scipy.linalg import expm


def _stoich(net):
    N, M = net.n_species, net.n_reactions
    R = np.zeros((M, N), dtype=np.int64)
    P = np.zeros((M, N), dtype=np.int64)
    for j in range(M):
        for s, c in net.reactants[j]:
            R[j, s] += c
        for s, c in net.products[j]:
            P[j, s] += c
    return R, P


def reachable_states(net, x0, cap=None, max_states=5000):
    """Breadth-first enumeration of the states reachable from x0; a species
    count above ``cap`` (open systems) is truncated away."""
    R, P = _stoich(net)
    nu = P - R
    start = tuple(int(v) for v in x0)
    seen = {start: 0}
    order = [start]
    q = [start]
    while q:
        x = q.pop()
        for j in range(net.n_reactions):
            if np.any(np.asarray(x) < R[j]):
                continue
            y = tuple(int(v) for v in np.asarray(x) + nu[j])
            if cap is not None and max(y) > cap:
                continue
            if y not in seen:
                seen[y] = len(order)
                order.append(y)
                q.append(y)
                if len(order) > max_states:
                    raise ValueError("state space too large")
    return order, seen


def generator(net, rates, states, index):
    R, P = _stoich(net)
    nu = P - R
    n = len(states)
    Q = np.zeros((n, n))
    for a, x in enumerate(states):
        xv = np.asarray(x)
        for j in range(net.n_reactions):
            h = 1
            for i in range(net.n_species):
                h *= comb(int(xv[i]), int(R[j, i]))
            prop = rates[j] * h
            if prop == 0:
                continue
            y = tuple(int(v) for v in xv + nu[j])
            if y not in index:
                continue  # truncated transition (open system)
            Q[a, index[y]] += prop
            Q[a, a] -= prop
    return Q


def distribution(net, rates, x0, t, cap=None):
    """Dict state -> probability at time t."""
    states, index = reachable_states(net, x0, cap=cap)
    Q = generator(net, rates, states, index)
    p0 = np.zeros(len(states))
    p0[0] = 1.0
    p = p0 @ expm(Q * t)
    return {s: float(v) for s, v in zip(states, p)}


def marginal(dist, species):
    out = {}
    for s, p in dist.items():
        out[s[species]] = out.get(s[species], 0.0) + p
    return out
