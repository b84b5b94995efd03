"""Seeded synthetic problem descriptions.

This module only builds *data*: geometry boxes, cross sections, sources,
tally meshes and run parameters, as plain Python dicts of numpy arrays.  It
contains none of the transport arithmetic.  Both the CPU oracle (under
``oracle/``) and the GPU library consume these dicts through their own,
separate marshalling code.

Problem dict schema (all lengths in cm, times in s):

``outer_lo``, ``outer_hi``   float64[3]; +-inf allowed (slab problems)
``bc``                       int[6] for faces -x,+x,-y,+y,-z,+z: 0 vacuum, 1 reflective
``box_lo``, ``box_hi``       float64[nb,3]; cells are priority-ordered boxes
``box_mat``                  int[nb]
``background_mat``           material outside every box
``sigma_t``                  float64[M,G]
``sigma_s``                  float64[M,G,G]; row = from group, column = to group
``speed``                    float64[G]
``source``                   dict(kind 'point'|'box', lo[3], hi[3], t0, t1,
                             isotropic, dir[3], group)
``mesh``                     dict(lo[4], hi[4], n[4], per_group); axes x,y,z,t.
                             An axis with lo=-inf and hi=+inf is unbounded (n=1).
``census``                   float64[nc] increasing census times; last = end time
``implicit_capture``         bool; ``w_cut``, ``w_surv`` for its weight cutoff
``detector``                 None or dict(lo[3], hi[3])
``n_batches``                batches for the mesh-tally statistics
``collision_tally``          bool; also score the collision estimator w/Sigma_t on the mesh
``surface_tally``            None or dict(axis, pos): also a surface-current tally on the
                             plane x[axis] = pos, binned by side of crossing, group (per-group
                             meshes), the mesh's time bins and its bins on the other two axes
``population_control``       None or dict(target): splitting-roulette of every intermediate
                             census bank to `target` particles per source history
``max_events``               flight cap per history
``stack_cap``                LIFO depth for split daughters per history
``importance``               None or dict(n[4]) coarse space-time grid
``ww``                       None or dict(params float32[...], hidden, logk, ratio, n_max,
                             ymin, ymax, map (nx, ny, nz, nt) or None)
``nu_sigma_f``, ``chi``      None, or float64[M,G] each: fission production nu*Sigma_f per
                             material and group, and the fission spectrum (outgoing group
                             of a fission neutron); problems with fission run in the
                             k-eigenvalue mode

The slab of the one-group problem is an outer box with infinite y/z extent; a
plane source on x=0 is then a point source at the origin (translation
invariance in y and z makes the two identical).
"""
from __future__ import annotations

import copy
import math

import numpy as np

INF = float("inf")
ROOT_SEED = 20260001

VACUUM = 0
REFLECTIVE = 1


def _base(G: int = 1) -> dict:
    return dict(
        outer_lo=np.zeros(3), outer_hi=np.ones(3), bc=np.zeros(6, np.int32),
        box_lo=np.zeros((0, 3)), box_hi=np.zeros((0, 3)), box_mat=np.zeros(0, np.int32),
        background_mat=0,
        sigma_t=np.ones((1, G)), sigma_s=np.zeros((1, G, G)), speed=np.ones(G),
        source=dict(kind="point", lo=np.zeros(3), hi=np.zeros(3), t0=0.0, t1=0.0,
                    isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=G - 1),
        mesh=dict(lo=np.array([0.0, -INF, -INF, 0.0]), hi=np.array([1.0, INF, INF, 1.0]),
                  n=np.array([1, 1, 1, 1], np.int32), per_group=False),
        census=np.array([1.0]),
        implicit_capture=False, w_cut=0.25, w_surv=1.0,
        detector=None, n_batches=20, max_events=1_000_000, stack_cap=64,
        importance=None, ww=None, collision_tally=False, surface_tally=None,
        population_control=None, nu_sigma_f=None, chi=None,
    )


def slab_problem(sigma_t=1.0, c=0.5, length=10.0, t_end=10.0, nx=100, nt=20, v=1.0,
                 isotropic=True, reflective=False, detector=(9.0, 10.0)) -> dict:
    """One-group slab [0, length] with infinite y/z extent, pulse at x=0, t=0."""
    p = _base(1)
    p["outer_lo"] = np.array([0.0, -INF, -INF])
    p["outer_hi"] = np.array([length, INF, INF])
    p["bc"] = np.full(6, REFLECTIVE if reflective else VACUUM, np.int32)
    p["sigma_t"] = np.array([[sigma_t]])
    p["sigma_s"] = np.array([[[c * sigma_t]]])
    p["speed"] = np.array([v])
    p["source"] = dict(kind="point", lo=np.zeros(3), hi=np.zeros(3), t0=0.0, t1=0.0,
                       isotropic=isotropic, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([0.0, -INF, -INF, 0.0]), hi=np.array([length, INF, INF, t_end]),
                     n=np.array([nx, 1, 1, nt], np.int32), per_group=False)
    p["census"] = np.array([t_end])
    if detector is not None:
        p["detector"] = dict(lo=np.array([detector[0], -INF, -INF]),
                             hi=np.array([detector[1], INF, INF]))
    return p


def config1() -> dict:
    """1D slab 0-10 cm, Sigma_t=1, c=0.5, v=1, pulsed isotropic plane source at
    x=0, t=0, vacuum; tally 100 x-bins by 20 t-bins over [0,10] s."""
    return slab_problem()


def infinite_medium(sigma_t, sigma_s, speed, half=50.0, t_end=10.0, nt=10,
                    src_group=None, implicit=False) -> dict:
    """All-reflective homogeneous box, pulse at the centre at t=0.  Used by the
    pulsed-decay pins (population exp(-v Sigma_a t) and its multigroup form)."""
    sigma_t = np.atleast_1d(np.asarray(sigma_t, float))
    G = sigma_t.size
    p = _base(G)
    p["outer_lo"] = np.full(3, -half)
    p["outer_hi"] = np.full(3, half)
    p["bc"] = np.full(6, REFLECTIVE, np.int32)
    p["sigma_t"] = sigma_t.reshape(1, G)
    p["sigma_s"] = np.asarray(sigma_s, float).reshape(1, G, G)
    p["speed"] = np.atleast_1d(np.asarray(speed, float))
    p["source"]["group"] = G - 1 if src_group is None else src_group
    p["mesh"] = dict(lo=np.array([-half, -half, -half, 0.0]), hi=np.array([half, half, half, t_end]),
                     n=np.array([1, 1, 1, nt], np.int32), per_group=G > 1)
    p["census"] = np.array([t_end])
    p["implicit_capture"] = implicit
    return p


# ---------------------------------------------------------------------------
# 3D duct stand-in (synthetic; not the published benchmark's coordinates)
# ---------------------------------------------------------------------------

SOURCE_CUBE = ([0.0, 0.0, 0.0], [10.0, 10.0, 10.0])
DUCT_LEGS = [
    ([0.0, 10.0, 0.0], [10.0, 50.0, 10.0]),     # leg 1: up +y out of the source cube
    ([10.0, 40.0, 0.0], [40.0, 50.0, 10.0]),    # leg 2: first right-angle turn, along +x
    ([30.0, 50.0, 0.0], [40.0, 100.0, 10.0]),   # leg 3: second turn, along +y to the y=100 face
]
DETECTOR = ([30.0, 90.0, 0.0], [40.0, 100.0, 10.0])   # last 10 cm of the duct, at its exit


def duct_geometry(p: dict) -> dict:
    boxes = [SOURCE_CUBE] + DUCT_LEGS
    p["outer_lo"] = np.array([0.0, 0.0, 0.0])
    p["outer_hi"] = np.array([60.0, 100.0, 60.0])
    p["bc"] = np.zeros(6, np.int32)
    p["box_lo"] = np.array([b[0] for b in boxes], float)
    p["box_hi"] = np.array([b[1] for b in boxes], float)
    p["box_mat"] = np.array([0, 1, 1, 1], np.int32)   # 0 source, 1 duct, 2 shield
    p["background_mat"] = 2
    p["detector"] = dict(lo=np.array(DETECTOR[0]), hi=np.array(DETECTOR[1]))
    return p


def config2(n_census: int = 1) -> dict:
    """3D box 60x100x60, one group, v=1; source cube Sigma_t=0.1, c=0.5, uniform
    isotropic source on t in [0,50]; bent 10x10 duct (Sigma_t=1e-4, c=0.5);
    shield Sigma_t=0.1, c=0.5; 1 cm mesh x 20 t-bins over [0,200] s."""
    p = duct_geometry(_base(1))
    p["sigma_t"] = np.array([[0.1], [1e-4], [0.1]])
    p["sigma_s"] = 0.5 * p["sigma_t"].reshape(3, 1, 1)
    p["speed"] = np.array([1.0])
    p["source"] = dict(kind="box", lo=np.array(SOURCE_CUBE[0]), hi=np.array(SOURCE_CUBE[1]),
                       t0=0.0, t1=50.0, isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([60.0, 100.0, 60.0, 200.0]),
                     n=np.array([60, 100, 60, 20], np.int32), per_group=False)
    p["census"] = np.linspace(0.0, 200.0, n_census + 1)[1:]
    return p


def config3(seed: int = ROOT_SEED, n_census: int = 1) -> dict:
    """Config-2 geometry with 7 groups.  Per region and group Sigma_t ~ U(0.05,0.5)
    and c ~ U(0.3,0.9); lower-triangular downscatter (to-group <= from-group,
    group 0 slowest) whose row sums are c*Sigma_t, off-diagonal split by
    normalised U(0,1) weights; speeds 10^(1+g/2) cm/s; source in the fastest group."""
    G = 7
    rng = np.random.default_rng(seed)
    p = duct_geometry(_base(G))
    st = rng.uniform(0.05, 0.5, size=(3, G))
    c = rng.uniform(0.3, 0.9, size=(3, G))
    ss = np.zeros((3, G, G))
    for m in range(3):
        for g in range(G):
            wts = rng.uniform(0.0, 1.0, size=g + 1)
            ss[m, g, : g + 1] = c[m, g] * st[m, g] * wts / wts.sum()
    p["sigma_t"] = st
    p["sigma_s"] = ss
    p["speed"] = 10.0 ** (1.0 + np.arange(G) / 2.0)
    p["source"] = dict(kind="box", lo=np.array(SOURCE_CUBE[0]), hi=np.array(SOURCE_CUBE[1]),
                       t0=0.0, t1=50.0, isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=G - 1)
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([60.0, 100.0, 60.0, 200.0]),
                     n=np.array([60, 100, 60, 20], np.int32), per_group=True)
    p["census"] = np.linspace(0.0, 200.0, n_census + 1)[1:]
    return p


def coarse_importance_grid() -> dict:
    """Coarse space-time grid (10 cm cells x 10 s) for importance estimation."""
    return dict(n=np.array([6, 10, 6, 20], np.int32))


def config4(ww: dict | None = None) -> dict:
    """Config-2 problem with learned weight windows attached (``ww``)."""
    p = config2()
    p["ww"] = ww
    return p


# ---------------------------------------------------------------------------
# Batched problems (256 uneven boxes)
# ---------------------------------------------------------------------------

def _bisect_regions(rng, lo, hi, n_regions):
    """Recursive axis-aligned bisection of [lo,hi] into n_regions boxes."""
    boxes = [(np.array(lo, float), np.array(hi, float))]
    while len(boxes) < n_regions:
        i = int(np.argmax([np.prod(b[1] - b[0]) for b in boxes]))
        blo, bhi = boxes.pop(i)
        ax = int(np.argmax(bhi - blo))
        cut = blo[ax] + rng.uniform(0.2, 0.8) * (bhi[ax] - blo[ax])
        h1 = bhi.copy(); h1[ax] = cut
        l2 = blo.copy(); l2[ax] = cut
        boxes += [(blo, h1), (l2, bhi)]
    return boxes


def batch_problem(seed: int, nt: int = 10, n_mesh: int = 20) -> dict:
    """One of the batched problems: box axes U(5,100) cm, 1-8 regions from a
    recursive bisection, Sigma_t ~ U(0.01,1), c ~ U(0,0.95), 1-7 groups
    (v=1 for one group, else log-spaced 1e1..1e4), isotropic point source at
    the centre at t=0 in the fastest group, end time 5*L_max/v_min split into
    ``nt`` census steps that coincide with the tally's time bins."""
    rng = np.random.default_rng(seed)
    L = rng.uniform(5.0, 100.0, size=3)
    n_reg = int(rng.integers(1, 9))
    G = int(rng.integers(1, 8))
    regions = _bisect_regions(rng, np.zeros(3), L, n_reg)
    st = rng.uniform(0.01, 1.0, size=(n_reg, G))
    c = rng.uniform(0.0, 0.95, size=(n_reg, G))
    ss = np.zeros((n_reg, G, G))
    for m in range(n_reg):
        for g in range(G):
            wts = rng.uniform(0.0, 1.0, size=g + 1)
            ss[m, g, : g + 1] = c[m, g] * st[m, g] * wts / wts.sum()
    speed = np.array([1.0]) if G == 1 else np.logspace(1.0, 4.0, G)
    t_end = 5.0 * float(L.max()) / float(speed.min())
    p = _base(G)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = L.copy()
    p["bc"] = np.zeros(6, np.int32)
    # the last region doubles as the background material; the others are boxes
    p["box_lo"] = np.array([r[0] for r in regions[:-1]], float).reshape(-1, 3)
    p["box_hi"] = np.array([r[1] for r in regions[:-1]], float).reshape(-1, 3)
    p["box_mat"] = np.arange(n_reg - 1, dtype=np.int32)
    p["background_mat"] = n_reg - 1
    p["sigma_t"] = st
    p["sigma_s"] = ss
    p["speed"] = speed
    p["source"] = dict(kind="point", lo=L / 2.0, hi=L / 2.0, t0=0.0, t1=0.0, isotropic=True,
                       dir=np.array([1.0, 0.0, 0.0]), group=G - 1)
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([L[0], L[1], L[2], t_end]),
                     n=np.array([n_mesh, n_mesh, n_mesh, nt], np.int32), per_group=False)
    p["census"] = np.linspace(0.0, t_end, nt + 1)[1:]
    p["detector"] = None
    p["n_batches"] = 1
    return p


def config5(n_problems: int = 256, seed: int = ROOT_SEED):
    """Batched workload: list of problem dicts and the histories per problem
    (log-uniform between 1e4 and 1e6)."""
    rng = np.random.default_rng(seed)
    n_hist = np.floor(10.0 ** rng.uniform(4.0, 6.0, size=n_problems)).astype(np.int64)
    probs = [batch_problem(seed + 1 + i) for i in range(n_problems)]
    return probs, n_hist


# ---------------------------------------------------------------------------
# k-eigenvalue problems (steady state: every generation starts at t = 0)
# ---------------------------------------------------------------------------

T_STEADY = 1.0e30          # one census edge far beyond any history


def keff_infinite_medium(sigma_t, sigma_s, nu_sigma_f, chi, half=50.0) -> dict:
    """Homogeneous all-reflective box with fission; the first generation
    starts at the centre in the fastest group.  Its multiplication is the
    infinite-medium k, a closed form of the data."""
    sigma_t = np.atleast_1d(np.asarray(sigma_t, float))
    G = sigma_t.size
    p = infinite_medium(sigma_t, sigma_s, np.ones(G), half=half, t_end=T_STEADY, nt=1)
    p["nu_sigma_f"] = np.asarray(nu_sigma_f, float).reshape(1, G)
    p["chi"] = np.asarray(chi, float).reshape(1, G)
    p["mesh"]["per_group"] = G > 1
    return p


CORE_HALF, REFLECTOR_HALF = 20.0, 30.0


def keff_core(nx: int = 30) -> dict:
    """Two-group reflected core (synthetic data, chosen for k near 1; not a
    published benchmark): a 40 cm fissile cube centred in a 60 cm cube of
    moderating reflector, vacuum outside.  Group 0 thermal, group 1 fast;
    every fission neutron is born fast.  Mesh nx^3 x 2 groups, one time bin;
    the first generation is a uniform source over the core."""
    G = 2
    p = _base(G)
    p["outer_lo"] = np.full(3, -REFLECTOR_HALF)
    p["outer_hi"] = np.full(3, REFLECTOR_HALF)
    p["bc"] = np.zeros(6, np.int32)
    p["box_lo"] = np.full((1, 3), -CORE_HALF)
    p["box_hi"] = np.full((1, 3), CORE_HALF)
    p["box_mat"] = np.array([0], np.int32)
    p["background_mat"] = 1
    #                 thermal  fast
    p["sigma_t"] = np.array([[1.25, 0.25],          # core
                             [1.50, 0.30]])         # reflector
    p["sigma_s"] = np.zeros((2, G, G))              # rows: from-group
    p["sigma_s"][0] = [[1.05, 0.0], [0.017, 0.205]]
    p["sigma_s"][1] = [[1.48, 0.0], [0.035, 0.264]]
    p["nu_sigma_f"] = np.array([[0.50, 0.008], [0.0, 0.0]])
    p["chi"] = np.array([[0.0, 1.0], [0.0, 1.0]])
    p["speed"] = np.array([2.2e5, 1.0e7])
    p["source"] = dict(kind="box", lo=np.full(3, -CORE_HALF), hi=np.full(3, CORE_HALF), t0=0.0,
                       t1=0.0, isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=1)
    p["mesh"] = dict(lo=np.array([-REFLECTOR_HALF] * 3 + [0.0]),
                     hi=np.array([REFLECTOR_HALF] * 3 + [T_STEADY]),
                     n=np.array([nx, nx, nx, 1], np.int32), per_group=True)
    p["census"] = np.array([T_STEADY])
    p["detector"] = dict(lo=np.full(3, -5.0), hi=np.full(3, 5.0))
    return p


def with_(p: dict, **kw) -> dict:
    """Deep copy of a problem with top-level keys replaced."""
    q = copy.deepcopy(p)
    q.update(kw)
    return q


def n_bins(p: dict) -> int:
    n = [int(v) for v in p["mesh"]["n"]]
    G = p["sigma_t"].shape[1] if p["mesh"]["per_group"] else 1
    return G * n[0] * n[1] * n[2] * n[3]


def mlp_param_count(in_dim: int, hidden: int = 64) -> int:
    return hidden * in_dim + hidden + hidden * hidden + hidden + hidden + 1
