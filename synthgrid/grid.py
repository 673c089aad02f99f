"""Seeded synthetic grids shaped like the paper's AC-OPF workloads.

The paper benchmarks MATPOWER cases (Table 1 of its numerical section) that are
not available here.  These generators draw stand-ins with the same bus, line and
generator counts and with the parameter distributions of the benchmark
configurations:

* topology: a spanning tree plus chords on a random geometric embedding (buses
  uniform in the unit square; every new bus attaches to one of its 3 nearest
  placed buses; chords join a bus to one of its 6 nearest non-adjacent buses),
  which keeps the graph near-planar like a real transmission grid;
* lines: r ~ U[0.01, 0.1], x ~ U[0.05, 0.4], total charging b ~ U[0, 0.05] (pu);
* loads: P ~ U[0.1, 0.5] pu, Q = 0.3 P;
* generators at distinct buses spread over the embedding (best of 4 random
  candidates by distance to the generators already placed); Pmax = (load of
  the buses nearest to the unit + a floor) * U[0.5, 1.5], rescaled to sum to
  twice the base load, plus recourse headroom max(1, 0.6 ||Pd||_2) on the
  largest unit (the reference bus, which balances every scenario), Pmin = 0, Q in +-0.5 Pmax, costs c2 ~ U[0.01, 0.1]
  $/MW^2h, c1 ~ U[10, 40] $/MWh, c0 = 0;
* voltage magnitude bounds [0.9, 1.1];
* line ratings from a DC flow estimate at proportional dispatch (see
  ``_line_ratings``), so that flow limits are meaningful but not binding
  everywhere;
* scenario load factors clip(1 + sigma * xi, 0.5, 1.5), xi ~ N(0, 1) iid per
  (load, scenario); Q scales with P.

All arrays are numpy, float64 values and int32 indices.  Per-scenario arrays
are laid out [n_load][N] (scenario index fastest).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class Network:
    n_bus: int
    n_line: int
    n_gen: int
    ref_bus: int
    line_from: np.ndarray
    line_to: np.ndarray
    r: np.ndarray
    x: np.ndarray
    b: np.ndarray
    rate: np.ndarray          # apparent-power limit per line, pu
    gen_bus: np.ndarray
    pmin: np.ndarray
    pmax: np.ndarray
    qmin: np.ndarray
    qmax: np.ndarray
    c2: np.ndarray            # $/MW^2h
    c1: np.ndarray            # $/MWh
    c0: np.ndarray            # $/h
    vmin: np.ndarray
    vmax: np.ndarray
    load_bus: np.ndarray
    pd: np.ndarray            # base active load, pu
    qd: np.ndarray            # base reactive load, pu
    xy: np.ndarray = field(repr=False)
    seed: int = 0

    @property
    def n_load(self) -> int:
        return int(self.load_bus.shape[0])

    @property
    def ref_gen(self) -> int:
        return int(np.nonzero(self.gen_bus == self.ref_bus)[0][0])


@dataclass
class Scenarios:
    pd: np.ndarray            # [n_load][N]
    qd: np.ndarray            # [n_load][N]
    sigma: float
    seed: int

    @property
    def n_scen(self) -> int:
        return int(self.pd.shape[1])


@dataclass
class Instance:
    name: str
    net: Network
    scen: Scenarios


def dims(n_bus: int, n_line: int, n_gen: int) -> dict:
    """Problem sizes of the reduced-space AC-OPF split (one scenario block).

    State x = (voltage angles of the non-reference buses, magnitudes of the
    buses without a generator); control u = (magnitudes of the generator buses,
    active output of the non-reference generators); inequalities = (reference
    output, reactive output of every generator, squared flow at both ends of
    every line).
    """
    return dict(n_x=2 * n_bus - n_gen - 1, n_u=2 * n_gen - 1,
                m=2 * n_line + n_gen + 1)


def _tree_and_chords(rng, xy, n_line):
    n = xy.shape[0]
    edges = set()
    adj = [set() for _ in range(n)]
    order = rng.permutation(n)
    placed = np.empty(n, dtype=np.int64)
    placed[0] = order[0]
    for t in range(1, n):
        i = order[t]
        cand = placed[:t]
        d2 = np.sum((xy[cand] - xy[i]) ** 2, axis=1)
        k = min(3, t)
        near = cand[np.argpartition(d2, k - 1)[:k]] if t > k else cand
        j = int(near[rng.integers(len(near))])
        e = (min(i, j), max(i, j))
        edges.add(e)
        adj[i].add(j)
        adj[j].add(i)
        placed[t] = i
    n_chord = n_line - (n - 1)
    if n_chord < 0:
        raise ValueError("n_line must be at least n_bus - 1")
    # 6 nearest neighbours of every bus (brute force in blocks; n <= ~20k)
    knn = np.empty((n, min(6, n - 1)), dtype=np.int64)
    blk = 1024
    for s0 in range(0, n, blk):
        s1 = min(n, s0 + blk)
        d2 = np.sum((xy[s0:s1, None, :] - xy[None, :, :]) ** 2, axis=2)
        d2[np.arange(s1 - s0), np.arange(s0, s1)] = np.inf
        kk = knn.shape[1]
        part = np.argpartition(d2, kk - 1, axis=1)[:, :kk]
        dd = np.take_along_axis(d2, part, axis=1)
        knn[s0:s1] = np.take_along_axis(part, np.argsort(dd, axis=1), axis=1)
    added = 0
    tries = 0
    while added < n_chord:
        tries += 1
        if tries > 200 * max(n_chord, 1) + 10000:
            raise RuntimeError("could not place the requested number of chords")
        a = int(rng.integers(n))
        cand = [int(c) for c in knn[a] if int(c) not in adj[a]]
        if not cand:
            continue
        c = cand[int(rng.integers(len(cand)))]
        e = (min(a, c), max(a, c))
        if e in edges:
            continue
        edges.add(e)
        adj[a].add(c)
        adj[c].add(a)
        added += 1
    e = np.array(sorted(edges), dtype=np.int64)
    # random orientation and random order of the line list
    flip = rng.random(len(e)) < 0.5
    f = np.where(flip, e[:, 1], e[:, 0])
    t = np.where(flip, e[:, 0], e[:, 1])
    perm = rng.permutation(len(e))
    return f[perm].astype(np.int32), t[perm].astype(np.int32)


def _spread_choice(rng, xy, k):
    """k distinct buses spread over the embedding: every next pick is the best
    of 4 random candidates by distance to the buses already picked."""
    n = xy.shape[0]
    first = int(rng.integers(n))
    chosen = [first]
    taken = np.zeros(n, dtype=bool)
    taken[first] = True
    dmin = np.sum((xy - xy[first]) ** 2, axis=1)
    for _ in range(k - 1):
        free = np.nonzero(~taken)[0]
        cand = free[rng.choice(len(free), size=min(4, len(free)), replace=False)]
        c = int(cand[np.argmax(dmin[cand])])
        chosen.append(c)
        taken[c] = True
        dmin = np.minimum(dmin, np.sum((xy - xy[c]) ** 2, axis=1))
    return np.array(chosen, dtype=np.int64)


def _nearest(pts, centres):
    out = np.empty(pts.shape[0], dtype=np.int64)
    for s0 in range(0, pts.shape[0], 2048):
        d2 = np.sum((pts[s0:s0 + 2048, None, :] - centres[None, :, :]) ** 2, axis=2)
        out[s0:s0 + 2048] = np.argmin(d2, axis=1)
    return out


def _line_ratings(rng, n_bus, ref, f, t, x, pinj):
    """DC-flow estimate of every line's flow, scaled into a rating.

    rating = max(0.3, U[1.5, 2.5] * |P_dc| + 0.1): a DC flow ignores reactive
    power and losses, so the margin is wider than a factor taken from an AC
    flow would be.
    """
    n_line = f.shape[0]
    bl = 1.0 / x
    rows = np.concatenate([f, t, f, t])
    cols = np.concatenate([f, t, t, f])
    vals = np.concatenate([bl, bl, -bl, -bl])
    B = sp.csr_matrix((vals, (rows, cols)), shape=(n_bus, n_bus))
    keep = np.array([i for i in range(n_bus) if i != ref])
    th = np.zeros(n_bus)
    th[keep] = spla.spsolve(B[keep][:, keep].tocsc(), pinj[keep])
    pf = (th[f] - th[t]) * bl
    return np.maximum(0.3, rng.uniform(1.5, 2.5, n_line) * np.abs(pf) + 0.1)


def make_network(n_bus: int, n_line: int, n_gen: int, seed: int,
                 loads="pq", load_scale: float = 1.0) -> Network:
    """Draw one connected grid.

    ``loads`` is "pq" (a load at every bus without a generator) or an integer
    count of distinct random load buses.  ``load_scale`` multiplies the drawn
    loads (a 9241-bus grid with these line impedances cannot carry U[0.1, 0.5]
    pu at every bus; its base-case power flow stops converging near 20% of it).
    """
    if n_gen < 1 or n_gen > n_bus:
        raise ValueError("need 1 <= n_gen <= n_bus")
    rng = np.random.default_rng(seed)
    xy = rng.random((n_bus, 2))
    f, t = _tree_and_chords(rng, xy, n_line)
    r = rng.uniform(0.01, 0.1, n_line)
    x = rng.uniform(0.05, 0.4, n_line)
    b = rng.uniform(0.0, 0.05, n_line)
    gen_bus = np.sort(_spread_choice(rng, xy, n_gen)).astype(np.int32)
    if loads == "pq":
        is_gen = np.zeros(n_bus, dtype=bool)
        is_gen[gen_bus] = True
        load_bus = np.nonzero(~is_gen)[0].astype(np.int32)
    else:
        load_bus = np.sort(rng.choice(n_bus, size=int(loads), replace=False)).astype(np.int32)
    pd = load_scale * rng.uniform(0.1, 0.5, load_bus.shape[0])
    qd = 0.3 * pd
    ptot = pd.sum()
    # capacity follows the load of each generator's neighbourhood (nearest
    # generator in the embedding), with a U[0.5, 1.5] spread, scaled so that
    # total capacity is twice the base load
    cell = np.zeros(n_gen)
    np.add.at(cell, _nearest(xy[load_bus], xy[gen_bus]), pd)
    pmax = (cell + 0.25 * ptot / n_gen) * rng.uniform(0.5, 1.5, n_gen)
    pmax *= 2.0 * ptot / pmax.sum()
    gref = int(np.argmax(pmax))
    # recourse headroom: about six standard deviations of the scenario total
    # load deviation at sigma = 0.1
    pmax[gref] += max(1.0, 0.6 * np.sqrt(np.sum(pd ** 2)))
    ref_bus = int(gen_bus[gref])
    pmin = np.zeros(n_gen)
    qmax = 0.5 * pmax
    qmin = -0.5 * pmax
    c2 = rng.uniform(0.01, 0.1, n_gen)
    c1 = rng.uniform(10.0, 40.0, n_gen)
    c0 = np.zeros(n_gen)
    vmin = np.full(n_bus, 0.9)
    vmax = np.full(n_bus, 1.1)
    pinj = np.zeros(n_bus)
    pdisp = pmax.copy()
    pdisp[gref] = np.median(pmax)
    np.add.at(pinj, gen_bus, pdisp * (ptot / pdisp.sum()))
    np.add.at(pinj, load_bus, -pd)
    rate = _line_ratings(rng, n_bus, ref_bus, f, t, x, pinj)
    return Network(n_bus=n_bus, n_line=n_line, n_gen=n_gen, ref_bus=ref_bus,
                   line_from=f, line_to=t, r=r, x=x, b=b, rate=rate,
                   gen_bus=gen_bus, pmin=pmin, pmax=pmax, qmin=qmin, qmax=qmax,
                   c2=c2, c1=c1, c0=c0, vmin=vmin, vmax=vmax,
                   load_bus=load_bus, pd=pd, qd=qd, xy=xy, seed=seed)


def make_scenarios(net: Network, n_scen: int, sigma: float, seed: int) -> Scenarios:
    """Load scenarios: base * clip(1 + sigma*xi, 0.5, 1.5), Q scaled with P."""
    rng = np.random.default_rng(seed)
    if sigma == 0.0:
        fac = np.ones((net.n_load, n_scen))
    else:
        fac = np.clip(1.0 + sigma * rng.standard_normal((net.n_load, n_scen)), 0.5, 1.5)
    pd = np.ascontiguousarray(net.pd[:, None] * fac)
    qd = np.ascontiguousarray(net.qd[:, None] * fac)
    return Scenarios(pd=pd, qd=qd, sigma=sigma, seed=seed)


# name -> (config number, n_bus, n_line, n_gen, N, loads, sigma, load scale,
#          accepted attempt)
PRESETS = {
    "c0": (0, 30, 41, 6, 1, "pq", 0.0, 1.0, 0),
    "c1": (1, 118, 186, 54, 128, 99, 0.1, 1.0, 0),
    "c3": (3, 118, 186, 54, 1, 99, 0.15, 1.0, 0),
    "c4": (4, 9241, 16049, 1445, 16, "pq", 0.1, 0.15, 0),
    "mid300": (92, 300, 450, 80, 4, "pq", 0.1, 1.0, 5),
    "tiny5": (90, 5, 6, 2, 2, "pq", 0.1, 1.0, 0),
    "tiny9": (91, 9, 12, 3, 3, "pq", 0.1, 1.0, 0),
}


def make_instance(n_bus, n_line, n_gen, n_scen, seed, loads="pq", sigma=0.1,
                  name="custom", load_scale=1.0) -> Instance:
    net = make_network(n_bus, n_line, n_gen, seed, loads, load_scale)
    scen = make_scenarios(net, n_scen, sigma, seed + 1)
    return Instance(name=name, net=net, scen=scen)


def preset(name: str, attempt: int | None = None, n_scen: int | None = None,
           sigma: float | None = None) -> Instance:
    """Named workload.  Grid seed = 1000*config + attempt, scenario seed = +1.

    c0: 30 buses / 41 lines / 6 generators, 1 scenario (loads at the 24 buses
        without a generator);
    c1: 118 / 186 / 54, 128 scenarios, 99 load buses, sigma 0.1 -- the sizes
        of the paper's case118;
    c3: the c1 grid with sigma 0.15 draws (warm-start training data);
    c4: 9241 / 16049 / 1445, 16 scenarios, loads (scaled by 0.15) at every
        bus without a generator -- the sizes of the paper's case9241pegase.

    ``attempt`` defaults to the accepted attempt of the table: the first whose
    base-case power flow converges and whose N = 1 interior-point solve
    converges (chosen by tests/golden/select_attempts.py).
    """
    cfg, nb, nl, ng, ns, loads, sg, lsc, acc = PRESETS[name]
    attempt = acc if attempt is None else attempt
    seed = 1000 * cfg + attempt
    if name == "c3":
        seed = 1000 * 1 + attempt   # same grid as c1
    inst = make_instance(nb, nl, ng, ns if n_scen is None else n_scen, seed,
                         loads=loads, sigma=sg if sigma is None else sigma,
                         name=name, load_scale=lsc)
    if name == "c3":
        inst.scen = make_scenarios(inst.net, inst.scen.n_scen, inst.scen.sigma,
                                   3000 + attempt + 1)
    return inst


def batch_instances(n: int = 64, seed: int = 2000, lo: int = 300, hi: int = 2000,
                    sigma: float = 0.1) -> list:
    """Independent single-scenario instances of uneven sizes: n_bus
    log-uniform in [lo, hi], n_line = round(1.5 n_bus), n_gen = round(0.15 n_bus),
    the parameter distributions of make_network."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nb = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        inst = make_instance(nb, int(round(1.5 * nb)), max(2, int(round(0.15 * nb))), 1,
                             seed * 1000 + i, loads="pq", sigma=sigma, name=f"batch{i}")
        out.append(inst)
    return out


def line_outages(net: Network, n_scen: int, seed: int, frac: float = 0.5) -> np.ndarray:
    """One tripped line or none per scenario (contingency scenarios): with
    probability `frac` a scenario trips a line drawn uniformly from the lines
    whose removal keeps the grid connected (so the state Jacobian stays
    nonsingular); -1 = no outage.  Seeded; no model arithmetic."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(seed)
    nb, nl = net.n_bus, net.n_line
    ok = []
    for l in range(nl):
        keep = np.arange(nl) != l
        f, t = net.line_from[keep], net.line_to[keep]
        adj = sp.coo_matrix((np.ones(len(f)), (f, t)), shape=(nb, nb))
        ncomp, _ = connected_components(adj, directed=False)
        if ncomp == 1:
            ok.append(l)
    ok = np.asarray(ok, dtype=np.int64)
    out = np.full(n_scen, -1, dtype=np.int64)
    trip = rng.uniform(size=n_scen) < frac
    out[trip] = rng.choice(ok, size=int(trip.sum()))
    return out
