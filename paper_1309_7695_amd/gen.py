"""Seeded synthetic inputs: reaction networks, rate constants, initial counts, sample times.

This module holds no arithmetic of the simulation method. It only draws the
inputs that both the HIP path and the CPU oracle consume, so that the two see
byte-identical arrays.

The problem statement these inputs instantiate is the paper's Methods section:
the state is a vector of molecule counts per species, reactions fire and change
it, and many independent simulations differ in their kinetic constants and
initial molecular amounts (Aims and motivation section). The paper's own model
(the Ras/cAMP/PKA pathway, Discussion section) is not reproduced; the seeded
networks below stand in for it.

Conventions
-----------
* A network is ``Network(n_species, reactants, products)`` where ``reactants[j]``
  and ``products[j]`` are lists of ``(species, coefficient)`` pairs, each species
  at most once per list.  Mass-action order (sum of reactant coefficients) is
  0, 1 or 2.
* Rates are float64 arrays of shape ``[M][T]`` (reaction-major, trajectory-minor).
* Initial counts are int32, either ``[N]`` (broadcast) or ``[N][T]``.
* Log-uniform on [a, b] means ``10 ** U(log10 a, log10 b)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Network:
    n_species: int
    reactants: list = field(default_factory=list)
    products: list = field(default_factory=list)
    name: str = ""

    @property
    def n_reactions(self) -> int:
        return len(self.reactants)

    def csr(self) -> dict:
        """Compressed-row arrays (int32) for reactants and products."""
        out = {}
        for tag, lists in (("react", self.reactants), ("prod", self.products)):
            ptr = [0]
            sp, co = [], []
            for lst in lists:
                for s, c in lst:
                    sp.append(int(s))
                    co.append(int(c))
                ptr.append(len(sp))
            out[tag + "_ptr"] = np.asarray(ptr, dtype=np.int32)
            out[tag + "_species"] = np.asarray(sp, dtype=np.int32)
            out[tag + "_coeff"] = np.asarray(co, dtype=np.int32)
        return out


def _canon(pairs):
    d = {}
    for s, c in pairs:
        d[int(s)] = d.get(int(s), 0) + int(c)
    return sorted(d.items())


def make_network(n_species, reactions, name=""):
    """reactions: list of (reactant_pairs, product_pairs)."""
    net = Network(n_species=n_species, name=name)
    for r, p in reactions:
        net.reactants.append(_canon(r))
        net.products.append(_canon(p))
    return net


# ----------------------------------------------------------------------------
# Small named networks (tests and the enzyme workload)
# ----------------------------------------------------------------------------

def enzyme_network():
    """E + S -> ES (k1), ES -> E + S (k-1), ES -> E + P (k2); species (E, S, ES, P)."""
    E, S, ES, P = 0, 1, 2, 3
    return make_network(4, [
        ([(E, 1), (S, 1)], [(ES, 1)]),
        ([(ES, 1)], [(E, 1), (S, 1)]),
        ([(ES, 1)], [(E, 1), (P, 1)]),
    ], name="enzyme")


def decay_network():
    """A -> 0."""
    return make_network(1, [([(0, 1)], [])], name="decay")


def birth_death_network():
    """0 -> A (k1), A -> 0 (k2)."""
    return make_network(1, [([], [(0, 1)]), ([(0, 1)], [])], name="birth_death")


def isomerization_network():
    """A -> B (k1), B -> A (k2)."""
    return make_network(2, [([(0, 1)], [(1, 1)]), ([(1, 1)], [(0, 1)])], name="isomerization")


def dimerization_network():
    """2A -> B."""
    return make_network(2, [([(0, 2)], [(1, 1)])], name="dimerization")


def source_network():
    """0 -> A."""
    return make_network(1, [([], [(0, 1)])], name="source")


def catalytic_network():
    """A -> A + B (A is a catalyst, never consumed)."""
    return make_network(2, [([(0, 1)], [(0, 1), (1, 1)])], name="catalytic")


def reversible_dimer_network():
    """2A -> B (k1), B -> 2A (k2): exercises the homodimer g_i rule both ways."""
    return make_network(2, [([(0, 2)], [(1, 1)]), ([(1, 1)], [(0, 2)])], name="reversible_dimer")


# ----------------------------------------------------------------------------
# Seeded random mass-action networks
# ----------------------------------------------------------------------------

def random_network(seed, n_species, n_reactions, frac_first=0.4, frac_second=0.5,
                   return_mass=False):
    """Random mass-action network with bounded mass.

    Reaction kinds: ``round(frac_first*M)`` first-order (one uniform reactant),
    ``round(frac_second*M)`` second-order (two reactant species drawn
    independently, so a homodimer occurs with probability 1/N), and the rest
    zero-order sources.  Products: 1 or 2 species drawn uniformly.  Every
    species carries a mass m_i ~ U{1,2,3}; a non-source reaction must satisfy
    sum(products m) <= sum(reactants m) (products are redrawn, and after 64
    failed draws the reaction becomes a pure degradation), which forbids
    runaway growth.  Null reactions (products == reactants) are redrawn.
    """
    rng = np.random.default_rng(seed)
    N, M = int(n_species), int(n_reactions)
    mass = rng.integers(1, 4, size=N)
    if not np.any(mass == 1):
        mass[rng.integers(N)] = 1
    n1 = int(round(frac_first * M))
    n2 = int(round(frac_second * M))
    n0 = M - n1 - n2
    kinds = np.array([1] * n1 + [2] * n2 + [0] * n0)
    kinds = kinds[rng.permutation(M)]
    reactions = []
    for j in range(M):
        kind = int(kinds[j])
        if kind == 0:
            react = []
        elif kind == 1:
            react = [(int(rng.integers(N)), 1)]
        else:
            a, b = (int(v) for v in rng.integers(N, size=2))
            react = [(a, 2)] if a == b else [(a, 1), (b, 1)]
        rmass = sum(int(mass[s]) * c for s, c in react)
        rc = _canon(react)
        prod = None
        for _ in range(64):
            npr = int(rng.integers(1, 3))
            sp = rng.integers(N, size=npr)
            cand = _canon([(int(s), 1) for s in sp])
            if kind != 0 and sum(int(mass[s]) * c for s, c in cand) > rmass:
                continue
            if cand == rc:
                continue
            prod = cand
            break
        if prod is None:
            prod = []
        reactions.append((react, prod))
    net = make_network(N, reactions, name=f"random_s{seed}_n{N}_m{M}")
    if return_mass:
        return net, mass
    return net


def log_uniform(rng, lo, hi, size):
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=size)


def sample_times(t_end, n_points):
    """Equally spaced sample times t_s = s*t_end/(n-1), the last one exactly t_end."""
    n = int(n_points)
    if n == 1:
        return np.array([float(t_end)])
    s = np.arange(n, dtype=np.float64)
    t = (s * float(t_end)) / float(n - 1)
    t[-1] = float(t_end)
    return t


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    net: Network
    rates: np.ndarray          # float64 [M][T]
    x0: np.ndarray             # int32 [N] (broadcast) or [N][T]
    times: np.ndarray          # float64 [S]
    eps: float = 0.03
    n_c: int = 10
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_traj(self):
        return self.rates.shape[1]


def enzyme_workload(n_traj=1024, seed=1):
    """Enzyme kinetics: x0 = (E, S, ES, P) = (100, 500, 0, 0); per-trajectory
    k1 ~ logU[1e-3, 1e-2], k-1 ~ logU[1e-2, 1e-1], k2 ~ logU[1e-2, 1e-1];
    t_end = 100 with 101 sample points."""
    rng = np.random.default_rng(seed)
    net = enzyme_network()
    rates = np.empty((3, n_traj))
    rates[0] = log_uniform(rng, 1e-3, 1e-2, n_traj)
    rates[1] = log_uniform(rng, 1e-2, 1e-1, n_traj)
    rates[2] = log_uniform(rng, 1e-2, 1e-1, n_traj)
    x0 = np.array([100, 500, 0, 0], dtype=np.int32)
    return Workload("enzyme_4x3", net, np.ascontiguousarray(rates), x0,
                    sample_times(100.0, 101), seed=seed)


def synthetic_workload(n_traj=65536, seed=2, n_species=50, n_reactions=100,
                       t_end=50.0, n_samples=200, rate_lo=1e-4, rate_hi=1.0,
                       low_count_frac=0.0):
    """Random 50-species, 100-reaction network from ``seed``: nominal rates
    logU[rate_lo, rate_hi], perturbed per trajectory by logU[0.1, 10];
    x0 ~ U{0..1000} drawn once and broadcast (a fraction ``low_count_frac`` of
    the species gets x0 ~ U{0..9} instead)."""
    net = random_network(seed, n_species, n_reactions)
    rng = np.random.default_rng(seed + 1_000_003)
    x0 = rng.integers(0, 1001, size=n_species).astype(np.int32)
    if low_count_frac > 0:
        k = int(round(low_count_frac * n_species))
        low = rng.permutation(n_species)[:k]
        x0[low] = rng.integers(0, 10, size=k)
    nominal = log_uniform(rng, rate_lo, rate_hi, n_reactions)
    pert = log_uniform(rng, 0.1, 10.0, (n_reactions, n_traj))
    rates = np.ascontiguousarray(nominal[:, None] * pert)
    return Workload(f"synthetic_{n_species}x{n_reactions}", net, rates, x0,
                    sample_times(t_end, n_samples), seed=seed)


def stiff_workload(n_traj=65536, seed=4):
    """Stiff multiscale network: 30 species, 80 reactions, nominal rates
    logU[1e-6, 1e2], 20% of species start below 10 molecules; t_end = 10,
    101 samples."""
    return synthetic_workload(n_traj=n_traj, seed=seed, n_species=30, n_reactions=80,
                              t_end=10.0, n_samples=101, rate_lo=1e-6, rate_hi=1e2,
                              low_count_frac=0.2)


def abundance_partition(net, x0, threshold=100):
    """Reaction partition for the hybrid sweep: reaction j is continuous (True)
    when every species it consumes or produces starts with at least
    ``threshold`` molecules, else discrete (a rule on the inputs only)."""
    cont = []
    for j in range(net.n_reactions):
        sp = {s for s, _ in net.reactants[j]} | {s for s, _ in net.products[j]}
        cont.append(all(int(x0[s]) >= threshold for s in sp))
    return np.array(cont, dtype=bool)


def hybrid_workload(n_traj=65536, seed=2, t_end=0.5, n_samples=11):
    """The 50x100 network of ``synthetic_workload`` with a fifth of its species
    starting below 10 molecules (the discrete part fires ~1,500 times per unit
    time per trajectory); pair it with ``abundance_partition``."""
    return synthetic_workload(n_traj=n_traj, seed=seed, t_end=t_end, n_samples=n_samples,
                              low_count_frac=0.2)


def int_log_uniform(rng, lo, hi, size=None):
    """Integers round(10^U(log10 lo, log10 hi)), clipped to [lo, hi]."""
    return np.clip(np.rint(log_uniform(rng, lo, hi, size)), lo, hi).astype(np.int64)


def batch_workloads(n_networks=64, seed=3000, m_range=(10, 500), t_range=(256, 16384),
                    t_end=50.0, n_samples=200, t_scale=1.0):
    """Uneven batch: network k from seed + k with M ~ integer logU[m_range] reactions
    and N = M // 2 species (same mix and rate/count distributions as the
    50x100 network), T_k ~ integer logU[t_range] trajectories (times t_scale,
    at least 1).  Sizes are drawn from a generator seeded with ``seed``."""
    rng = np.random.default_rng(seed)
    ms = int_log_uniform(rng, m_range[0], m_range[1], n_networks)
    ts = int_log_uniform(rng, t_range[0], t_range[1], n_networks)
    out = []
    for k in range(n_networks):
        m = int(ms[k])
        n_traj = max(1, int(round(ts[k] * t_scale)))
        w = synthetic_workload(n_traj=n_traj, seed=seed + k, n_species=max(m // 2, 1),
                               n_reactions=m, t_end=t_end, n_samples=n_samples)
        out.append(w)
    return out


def serve_specs(n_jobs=1050, seed=5000, rate=50.0, m_range=(20, 300), t_range=(1024, 65536),
                t_end_range=(10.0, 500.0), n_samples=101, t_scale=1.0, t_end_scale=1.0):
    """Serving stream: arrival times of a Poisson process of `rate` jobs/s
    (generator seed 5) and, per job k, (seed + k, M, T, t_end, n_samples) with
    M ~ integer logU[m_range] reactions, T ~ integer logU[t_range] trajectories
    (times t_scale) and t_end ~ logU[t_end_range] (times t_end_scale)."""
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
    srng = np.random.default_rng(seed)
    ms = int_log_uniform(srng, m_range[0], m_range[1], n_jobs)
    ts = int_log_uniform(srng, t_range[0], t_range[1], n_jobs)
    ends = log_uniform(srng, t_end_range[0], t_end_range[1], n_jobs)
    specs = [(seed + k, int(ms[k]), max(1, int(round(ts[k] * t_scale))),
              float(ends[k]) * t_end_scale, n_samples) for k in range(n_jobs)]
    return arrivals, specs


def serve_job(spec):
    """The workload of one serving-stream spec: the network of its seed with
    N = M // 2 species (mix and distributions of the 50x100 network)."""
    seed, m, n_traj, t_end, n_samples = spec
    return synthetic_workload(n_traj=n_traj, seed=seed, n_species=max(m // 2, 1),
                              n_reactions=m, t_end=t_end, n_samples=n_samples)


def serve_jobs(n_jobs=1050, **kw):
    """(arrival times, workloads) of the serving stream, built eagerly."""
    arrivals, specs = serve_specs(n_jobs=n_jobs, **kw)
    return arrivals, [serve_job(sp) for sp in specs]


def workload(name, n_traj=None):
    if name in ("enzyme", "enzyme_4x3"):
        return enzyme_workload(n_traj or 1024)
    if name in ("synthetic", "synthetic_50x100"):
        return synthetic_workload(n_traj or 65536)
    if name in ("stiff", "stiff_30x80"):
        return stiff_workload(n_traj or 65536)
    raise KeyError(name)
