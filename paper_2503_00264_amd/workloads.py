"""Seeded synthetic slab problems (inputs only).

This module draws the material data, cell widths, sources and time-step
settings of the slab transport problems that exercise the one-cell-inversion
(OCI) and source-iteration (SI) solvers.  It holds none of the method's
arithmetic: no discretisation, no quadrature, no solve.  The GPU library and
the tests' independent CPU reference are fed from the same arrays built here.

Every problem is a dict of plain numpy arrays (float64 unless noted):

  J, N, G        int   cells, Gauss-Legendre angles (even), energy groups
  dx             [J]           cell widths (cm)
  sigma_t        [J][G]        total cross section (1/cm)
  sigma_s        [J][G][G]     sigma_s[j][g][gp] = scattering gp -> g (1/cm)
  speed          [G]           particle speed (cm/s)
  dt             float         time-step size (s)
  steps          int           number of time steps
  q              [J][G][4]     isotropic source at (k,L), (k,R), (k+1/2,L), (k+1/2,R)
  inc_left       None          vacuum (prescribed incident flux of zero)
  inc_right      None
  psi_init       [J][G][N][2]  initial angular flux (L, R corners)

Recipes (the paper's problem family: slab geometry, vacuum boundaries,
isotropic source, zero initial flux, Gauss-Legendre S_N; section "Performance
on GPUs" and the scattering-ratio/optical-thickness sweeps of the Fourier
results section):

  homogeneous   one material, uniform cells, Q=1 everywhere.
  regions       R regions of equal cell count; per region sigma_t ~ U[0.1, 10]
                and scattering ratio c ~ U[0.5, 0.999] (one group), drawn in
                that order from numpy's PCG64 with the given seed; Q=1 in the
                first eighth of the regions.
  multigroup    as `regions` but G groups with a full scattering matrix:
                sigma_t[r][g] ~ U[0.1, 10]; for each source group gp a total
                ratio c ~ U[0.5, 0.999]; down-scatter gp->g>gp ~ U[0, 0.5]
                sigma_t[gp], up-scatter gp->g<gp ~ U[0, 0.05] sigma_t[gp];
                off-diagonal column sums above 0.9 c sigma_t[gp] are scaled
                down to 0.9 c sigma_t[gp]; the within-group term takes the
                rest, so each column sums to c sigma_t[gp] < sigma_t[gp].
  rosa          the paper's two-group test problem (its Table 2, physical
                reading of the scattering entries).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "homogeneous", "regions", "multigroup", "batch", "rosa",
    "config", "CONFIG_NAMES",
]


def _problem(dx, sigma_t, sigma_s, speed, dt, steps, q, N):
    J, G = sigma_t.shape
    return dict(
        J=int(J), N=int(N), G=int(G),
        dx=np.ascontiguousarray(dx, dtype=np.float64),
        sigma_t=np.ascontiguousarray(sigma_t, dtype=np.float64),
        sigma_s=np.ascontiguousarray(sigma_s, dtype=np.float64),
        speed=np.ascontiguousarray(speed, dtype=np.float64),
        dt=float(dt), steps=int(steps),
        q=np.ascontiguousarray(q, dtype=np.float64),
        inc_left=None, inc_right=None,
        psi_init=np.zeros((J, G, N, 2), dtype=np.float64),
    )


def homogeneous(J=64, N=8, length=4.0, sigma_t=1.0, c=0.9, speed=1.0,
                dt=0.1, steps=10, q=1.0):
    """One group, one material, uniform mesh on [0, length], source q everywhere."""
    dx = np.full(J, length / J)
    st = np.full((J, 1), sigma_t)
    ss = np.full((J, 1, 1), c * sigma_t)
    qq = np.full((J, 1, 4), q)
    return _problem(dx, st, ss, np.array([speed]), dt, steps, qq, N)


def regions(seed, J=4096, N=16, n_regions=64, length=64.0, speed=1.0,
            dt=0.1, steps=20, source_regions=None):
    """One group, `n_regions` random materials of J/n_regions cells each."""
    if J % n_regions:
        raise ValueError("J must be a multiple of n_regions")
    rng = np.random.default_rng(seed)
    st_r = rng.uniform(0.1, 10.0, size=n_regions)
    c_r = rng.uniform(0.5, 0.999, size=n_regions)
    per = J // n_regions
    reg = np.arange(J) // per
    dx = np.full(J, length / J)
    st = st_r[reg][:, None]
    ss = (c_r * st_r)[reg][:, None, None]
    nsrc = max(1, n_regions // 8) if source_regions is None else source_regions
    qq = np.zeros((J, 1, 4))
    qq[reg < nsrc] = 1.0
    return _problem(dx, st, ss, np.array([speed]), dt, steps, qq, N)


def _scatter_matrix(rng, st_g):
    """Draw one region's G x G scattering matrix, [g][gp] = gp -> g."""
    G = st_g.shape[0]
    ss = np.zeros((G, G))
    for gp in range(G):
        c_tot = rng.uniform(0.5, 0.999)
        col = np.zeros(G)
        for g in range(G):
            if g > gp:
                col[g] = rng.uniform(0.0, 0.5) * st_g[gp]
            elif g < gp:
                col[g] = rng.uniform(0.0, 0.05) * st_g[gp]
        off = col.sum()
        cap = 0.9 * c_tot * st_g[gp]
        if off > cap:
            col *= cap / off
            off = col.sum()
        col[gp] = c_tot * st_g[gp] - off
        ss[:, gp] = col
    return ss


def multigroup(seed, J=8192, N=16, G=4, n_regions=64, length=64.0,
               speeds=(1e3, 1e2, 10.0, 1.0), dt=1e-3, steps=10,
               source_regions=None):
    """G groups, `n_regions` random materials with full scattering matrices."""
    if J % n_regions:
        raise ValueError("J must be a multiple of n_regions")
    if len(speeds) < G:
        raise ValueError("need one speed per group")
    rng = np.random.default_rng(seed)
    st_r = rng.uniform(0.1, 10.0, size=(n_regions, G))
    ss_r = np.stack([_scatter_matrix(rng, st_r[r]) for r in range(n_regions)])
    per = J // n_regions
    reg = np.arange(J) // per
    dx = np.full(J, length / J)
    nsrc = max(1, n_regions // 8) if source_regions is None else source_regions
    qq = np.zeros((J, G, 4))
    qq[reg < nsrc] = 1.0
    sp = np.asarray(speeds[len(speeds) - G:], dtype=np.float64)
    return _problem(dx, st_r[reg], ss_r[reg], sp, dt, steps, qq, N)


def batch(seed=5, n_slabs=64, j_range=(256, 8192), n_choices=(8, 16, 32),
          g_choices=(1, 2, 4), dt=1e-3, steps=10, n_regions=64):
    """Independent slabs of uneven size; slab i draws from default_rng([seed, i]).

    Cell width 1/64 cm; region r holds the cells with floor(64 j / J) == r;
    one-group slabs follow `regions`, multigroup slabs `multigroup`, with the
    speeds being the last G entries of (1e3, 1e2, 10, 1).
    """
    slabs = []
    for i in range(n_slabs):
        rng = np.random.default_rng([seed, i])
        J = int(rng.integers(j_range[0], j_range[1] + 1))
        N = int(rng.choice(n_choices))
        G = int(rng.choice(g_choices))
        reg = (n_regions * np.arange(J)) // J
        st_r = rng.uniform(0.1, 10.0, size=(n_regions, G))
        if G == 1:
            c_r = rng.uniform(0.5, 0.999, size=n_regions)
            ss_r = (c_r * st_r[:, 0])[:, None, None]
        else:
            ss_r = np.stack([_scatter_matrix(rng, st_r[r]) for r in range(n_regions)])
        qq = np.zeros((J, G, 4))
        qq[reg < n_regions // 8] = 1.0
        sp = np.asarray((1e3, 1e2, 10.0, 1.0)[4 - G:], dtype=np.float64)
        slabs.append(_problem(np.full(J, 1.0 / 64.0), st_r[reg], ss_r[reg],
                              sp, dt, steps, qq, N))
    return slabs


# The smaller of the two total cross sections (group 2), 1/cm: the paper
# states the cell optical thickness delta of this problem with it.
ROSA_SIGMA_MIN = 0.45468
ROSA_LENGTH = 100.0


def rosa(J=1000, N=8, length=ROSA_LENGTH, dt=0.1, steps=1):
    """The paper's two-group test problem (Table 2), vacuum, Q=1, zero start."""
    st = np.array([1.5454, 0.45468])
    # [g][gp] = gp -> g : within-group 0.61789 / 0.0072534, 1->2 0.92747, 2->1 0.38211
    ss = np.array([[0.61789, 0.38211],
                   [0.92747, 0.0072534]])
    dx = np.full(J, length / J)
    qq = np.ones((J, 2, 4))
    return _problem(dx, np.tile(st, (J, 1)), np.tile(ss, (J, 1, 1)),
                    np.array([1.0, 0.5]), dt, steps, qq, N)


def fourier_verification(seed=2025, J=1000, N=8):
    """The paper's Fourier verification problem (section 3.1): 100 cm, vacuum,
    Sigma = 2.5/cm, dx = 0.1 cm, c = 0.9, dt = 0.1 s, v = 4 (read as cm/s,
    which gives the stated tau = 1), no source, S8, and a uniform [0, 1]
    random start for the angular flux."""
    p = homogeneous(J=J, N=N, length=0.1 * J, sigma_t=2.5, c=0.9, speed=4.0, dt=0.1, steps=1,
                    q=0.0)
    p["psi_init"] = np.random.default_rng(seed).uniform(0.0, 1.0, size=(J, 1, N, 2))
    return p


CONFIG_NAMES = ("homogeneous64", "regions4096", "multigroup8192",
                "multigroup16384", "batch64")

# Time-step sweep for the 4096-cell one-group problem, in mean free times of a
# reference 1/cm material at v = 1 cm/s, i.e. seconds.
REGIONS_DT_SWEEP = (1e-1, 1e-2, 1e-3, 1e-4)


def config(name, **over):
    """The five named workloads at full size (keyword overrides allowed)."""
    if name == "homogeneous64":
        return homogeneous(**over)
    if name == "regions4096":
        kw = dict(seed=2, J=4096, N=16, dt=1e-1, steps=20)
        kw.update(over)
        return regions(**kw)
    if name == "multigroup8192":
        kw = dict(seed=3, J=8192, N=16, G=4, dt=1e-3, steps=10)
        kw.update(over)
        return multigroup(**kw)
    if name == "multigroup16384":
        kw = dict(seed=4, J=16384, N=16, G=4, dt=1e-3, steps=20)
        kw.update(over)
        return multigroup(**kw)
    if name == "batch64":
        kw = dict(seed=5)
        kw.update(over)
        return batch(**kw)
    raise KeyError(name)
