"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws numbers: it holds none of the search method's arithmetic
(no envelope, no bound, no warping distance).  Every generator takes an explicit
seed tuple and returns float64 arrays; callers cast to float32 for the device.

Workloads (each stands in for a data set of the paper's experiments, Sec. 10):

* ``random_walk``: x_1 = 0 and x_i = x_{i-1} + N(0,1) (Sec. 10.1, also App. B).
  A series of length n holds the start value and n-1 Gaussian steps.
* ``shape_signatures``: centroid-distance signatures of random star-shaped
  polygons, a synthetic stand-in for the shape archives of Sec. 10.2, which are
  not available here.
* ``poisson_arrivals``: request arrival times for the serving loop.
* ``make_ragged_workload``: a batch of random-walk queries of mixed lengths and
  bands, each length with its own database (uneven batches; not a paper experiment).
* ``make_serving_workload``: a request stream over two resident databases (serving;
  not a paper experiment).
* ``triangle_triples``: independent triples of random walks or white noise (App. B).

Seeds follow ``SeedSequence([8113301, config_id, role, *extra])``, role 0 = database,
1 = queries, 2 = arrivals and per-request draws.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import convolve1d

BASE_SEED = 8113301

ROLE_DB = 0
ROLE_QUERY = 1
ROLE_ARRIVAL = 2


def rng(config_id: int, role: int, *extra: int) -> np.random.Generator:
    """PCG64 generator for (config, role, extra...)."""
    ss = np.random.SeedSequence([BASE_SEED, int(config_id), int(role), *[int(e) for e in extra]])
    return np.random.Generator(np.random.PCG64(ss))


def random_walk(count: int, n: int, gen: np.random.Generator) -> np.ndarray:
    """``count`` random walks of length ``n``: first value 0, then cumulative N(0,1) steps."""
    out = np.zeros((count, n), dtype=np.float64)
    if n > 1 and count > 0:
        steps = gen.standard_normal((count, n - 1))
        np.cumsum(steps, axis=1, out=out[:, 1:])
    return out


def white_noise(count: int, n: int, gen: np.random.Generator) -> np.ndarray:
    """``count`` series of i.i.d. N(0,1) values (App. B workload)."""
    return gen.standard_normal((count, n))


def _outlines(n: int, v: np.ndarray, theta: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Distance to the area centroid of n boundary points of each star-shaped polygon (v[c]
    vertices at sorted angles theta[c, :v[c]] and radii r[c, :v[c]]), spaced uniformly in arc
    length from vertex 0."""
    count, V = theta.shape
    i = np.arange(V)[None, :]
    live = i < v[:, None]
    nxt = np.where(i + 1 < v[:, None], i + 1, 0)
    px = np.where(live, r * np.cos(theta), 0.0)
    py = np.where(live, r * np.sin(theta), 0.0)
    qx = np.take_along_axis(px, nxt, axis=1)
    qy = np.take_along_axis(py, nxt, axis=1)
    cross = np.where(live, px * qy - qx * py, 0.0)
    area = 0.5 * cross.sum(axis=1)
    tiny = np.abs(area) < 1e-12
    safe = np.where(tiny, 1.0, area)
    cx = np.where(tiny, px.sum(axis=1) / v, ((px + qx) * cross).sum(axis=1) / (6.0 * safe))
    cy = np.where(tiny, py.sum(axis=1) / v, ((py + qy) * cross).sum(axis=1) / (6.0 * safe))
    seg = np.where(live, np.hypot(qx - px, qy - py), 0.0)
    cum = np.concatenate([np.zeros((count, 1)), np.cumsum(seg, axis=1)], axis=1)   # [count][V+1]
    s = np.arange(n)[None, :] * (cum[:, -1:] / n)                                    # [count][n]
    k = (cum[:, None, 1:] <= s[:, :, None]).sum(axis=2)                              # segment of each point
    k = np.minimum(k, v[:, None] - 1)
    segk = np.take_along_axis(seg, k, axis=1)
    t = (s - np.take_along_axis(cum, k, axis=1)) / np.where(segk > 0, segk, 1.0)
    pxk, pyk = np.take_along_axis(px, k, axis=1), np.take_along_axis(py, k, axis=1)
    bx = pxk + t * (np.take_along_axis(qx, k, axis=1) - pxk)
    by = pyk + t * (np.take_along_axis(qy, k, axis=1) - pyk)
    return np.hypot(bx - cx[:, None], by - cy[:, None])


def shape_signatures(count: int, n: int, gen: np.random.Generator, sigma: float = 4.0) -> np.ndarray:
    """``count`` z-normalised centroid-distance signatures of random star-shaped polygons:
    5..12 vertices at sorted uniform angles with radii U(0.5, 1.5); the distance of the
    outline to the area centroid (shoelace formula) at n points spaced uniformly in arc
    length, circularly smoothed by a Gaussian of ``sigma`` samples, then rotated by a random
    shift.  Draws, for all series at once: vertex counts, 12 angles and 12 radii per series
    (the first v used), shifts."""
    V = 12
    v = gen.integers(5, 13, count)                                  # 5..12 vertices
    theta = np.sort(np.where(np.arange(V)[None, :] < v[:, None],
                             gen.uniform(0.0, 2.0 * np.pi, (count, V)), np.inf), axis=1)
    theta = np.where(np.isfinite(theta), theta, 0.0)
    r = gen.uniform(0.5, 1.5, (count, V))
    shift = gen.integers(0, n, count)
    sig = np.empty((count, n))
    for c0 in range(0, count, 2048):
        c1 = min(count, c0 + 2048)
        sig[c0:c1] = _outlines(n, v[c0:c1], theta[c0:c1], r[c0:c1])
    if sigma > 0:  # circular Gaussian smoothing (wrap-around)
        half = int(np.ceil(4 * sigma))
        taps = np.arange(-half, half + 1)
        kern = np.exp(-0.5 * (taps / sigma) ** 2)
        kern /= kern.sum()
        sig = convolve1d(sig, kern, axis=1, mode="wrap")
    cols = (np.arange(n)[None, :] - shift[:, None]) % n   # rotate row c right by shift[c]
    sig = np.take_along_axis(sig, cols, axis=1)
    mean = sig.mean(axis=1, keepdims=True)
    sd = sig.std(axis=1, keepdims=True)
    return (sig - mean) / np.where(sd > 0, sd, 1.0)


def poisson_arrivals(rate_qps: float, count: int, gen: np.random.Generator) -> np.ndarray:
    """Arrival times (seconds from 0) of ``count`` requests of a Poisson process."""
    return np.cumsum(gen.exponential(1.0 / rate_qps, count))


def band_from_fraction(n: int, f: float) -> int:
    """Half-width w = floor(f*n + 0.5) for a band given as a fraction of the length."""
    return int(np.floor(f * n + 0.5))


# Named workloads: (database size, series length, query count, bands, exponents).
WORKLOADS = {
    "rw128_small": dict(config_id=1, N=1000, n=128, Q=16, w=(13,), p=(1,), kind="random_walk"),
    "rw256": dict(config_id=2, N=100_000, n=256, Q=256, w=(26,), p=(1, 2), kind="random_walk"),
    "shape512": dict(config_id=3, N=50_000, n=512, Q=512, w=(26, 51), p=(1,), kind="shape"),
}


def make_workload(name: str, N: int | None = None, Q: int | None = None):
    """Database and queries (float64) of a named workload, optionally truncated to N / Q."""
    spec = WORKLOADS[name]
    n = spec["n"]
    N = spec["N"] if N is None else N
    Q = spec["Q"] if Q is None else Q
    if spec["kind"] == "random_walk":
        db = random_walk(N, n, rng(spec["config_id"], ROLE_DB))
        qs = random_walk(Q, n, rng(spec["config_id"], ROLE_QUERY))
    else:
        db = shape_signatures(N, n, rng(spec["config_id"], ROLE_DB))
        qs = shape_signatures(Q, n, rng(spec["config_id"], ROLE_QUERY))
    return db, qs


def triangle_triples(count: int = 100_000, n: int = 100, kind: str = "random_walk", config_id: int = 6):
    """``count`` triples (x, y, z) of independent series of length n (App. B experiment: random
    walks or white noise, 100,000 triples of 100 samples).  Returns three [count][n] arrays."""
    draw = random_walk if kind == "random_walk" else white_noise
    role = 0 if kind == "random_walk" else 1
    return tuple(draw(count, n, rng(config_id, role, j)) for j in range(3))


RAGGED_LENGTHS = (64, 128, 256, 512, 1024)
RAGGED_FRACTIONS = (0.05, 0.1, 0.2)


def make_ragged_workload(Q: int = 4096, N: int = 20_000, lengths=RAGGED_LENGTHS, fractions=RAGGED_FRACTIONS,
                         config_id: int = 4):
    """Uneven batch: Q random-walk queries, length uniform over ``lengths``, band
    w = round(f * n) with f uniform over ``fractions``; one random-walk database of N
    series per length.  Returns (dbs, queries, db_of, w): dbs[i] is [N][lengths[i]],
    queries a list of 1-D arrays, db_of[q] the database of query q."""
    r = rng(config_id, ROLE_QUERY)
    db_of = r.integers(0, len(lengths), Q).astype(np.int32)
    frac = r.integers(0, len(fractions), Q)
    w = np.array([band_from_fraction(lengths[b], fractions[f]) for b, f in zip(db_of, frac)], dtype=np.int32)
    dbs = [random_walk(N, n, rng(config_id, ROLE_DB, i)) for i, n in enumerate(lengths)]
    queries = [None] * Q
    for i, n in enumerate(lengths):
        sel = np.nonzero(db_of == i)[0]
        qs = random_walk(len(sel), n, rng(config_id, ROLE_QUERY, 1, i))
        for j, q in enumerate(sel):
            queries[q] = qs[j]
    return dbs, queries, db_of, w


def make_serving_workload(rate_qps: float, count: int, N_main: int = 1_000_000, N_side: int = 200_000,
                          n_main: int = 128, n_side: int = 256, side_share: float = 0.2, ks=(1, 5, 10),
                          f: float = 0.1, config_id: int = 5, with_databases: bool = True):
    """Request stream for the serving loop: ``count`` Poisson arrivals at ``rate_qps``; each
    request asks the main database (length n_main) or, with probability side_share, the side
    database (length n_side), with w = round(f * n) and k drawn uniformly from ``ks``.
    Returns (dbs, requests) with dbs = [main, side] random-walk databases (None when
    with_databases is false) and requests a dict of arrays: t (s), db, w, k and the list
    ``y`` of query series."""
    r = rng(config_id, ROLE_ARRIVAL, int(rate_qps))
    t = poisson_arrivals(rate_qps, count, r)
    db = (r.random(count) < side_share).astype(np.int32)
    k = np.asarray(ks, dtype=np.int32)[r.integers(0, len(ks), count)]
    lengths = (n_main, n_side)
    w = np.array([band_from_fraction(lengths[b], f) for b in db], dtype=np.int32)
    yq = random_walk(count, n_side, rng(config_id, ROLE_QUERY, int(rate_qps)))
    y = [yq[i, :lengths[b]] for i, b in enumerate(db)]
    dbs = None
    if with_databases:
        dbs = [random_walk(N_main, n_main, rng(config_id, ROLE_DB, 0)),
               random_walk(N_side, n_side, rng(config_id, ROLE_DB, 1))]
    return dbs, dict(t=t, db=db, w=w, k=k, y=y)
