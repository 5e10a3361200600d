"""Seeded synthetic inputs for fast-FCM mobility evaluations.

This module only draws inputs (positions, forces, torques) and states the run
parameters of each workload; it holds none of the method's arithmetic and is
shared by the tests, the benchmark and the oracle-side checks alike.  The paper
measures on random suspensions (Sec. 5.1-5.3) and on sedimenting rods
(Sec. 6.1); these generators stand in for them.

Random numbers: numpy's PCG64 generator seeded with 231012651 + workload index,
drawing positions first, then forces, then torques.  "Non-overlapping" means
random sequential addition: uniform proposals rejected when the minimum-image
distance to an already placed centre is below 2a.

Workloads (a = 1, eta = 1, sigma = a / sqrt(pi)):

  0  small    N = 64, L = 40, grid 32^3, Sigma = 2 sigma, M_G = 12,
              R_c = 10.800045715206082 (the radius beyond which every scaled
              correction entry is < 1e-10; value printed by
              ``python -m oracle.derive``); net force removed.
  1  dilute   N = 10^4, volume fraction 1 %, grid 128^3, Sigma = dx, M_G = 10,
              R_c = 5.5 Sigma.
  2  dense    N = 10^5, volume fraction 10 %, grid 256^3, Sigma = dx,
              M_G = 10, R_c = 5.5 Sigma.
  3  rods     2000 rigid rods of 30 touching spheres (N = 60000) in one half
              of a periodic cube L = 600, grid 192^3, Sigma = dx, M_G = 10,
              R_c = 5.5 Sigma; F = x^ + N(0, 0.1^2) per component, T = 0.

The serving stream is drawn by ``serving_stream`` (positions of its requests
by ``lattice_positions``: non-overlapping, drawn fast enough for 512 requests).
"""

import math

import numpy as np

SEED_BASE = 231012651
C1_RCUT = 10.800045715206082


def rng_for(index):
    return np.random.default_rng(SEED_BASE + int(index))


class _Cells:
    """Uniform cell grid of width >= 2a used only to reject overlaps."""

    def __init__(self, L, a):
        self.L = L
        self.m = max(int(L / (2.0 * a)), 1)
        self.w = L / self.m
        self.cells = {}
        self.a2 = (2.0 * a) ** 2

    def _key(self, p):
        c = np.floor(p / self.w).astype(np.int64) % self.m
        return int(c[0]), int(c[1]), int(c[2])

    def overlaps(self, p):
        cx, cy, cz = self._key(p)
        m, L = self.m, self.L
        rng = (-1, 0, 1) if m >= 3 else range(-(m // 2), m - m // 2)
        for ox in rng:
            for oy in rng:
                for oz in rng:
                    lst = self.cells.get(((cx + ox) % m, (cy + oy) % m, (cz + oz) % m))
                    if not lst:
                        continue
                    q = np.asarray(lst)
                    d = p[None, :] - q
                    d -= L * np.round(d / L)
                    if np.any(np.sum(d * d, axis=1) < self.a2 * (1.0 - 1e-12)):
                        return True
        return False

    def add(self, p):
        self.cells.setdefault(self._key(p), []).append(p.copy())


def rsa_positions(N, L, a, rng, max_tries=200):
    """Random sequential addition of N non-overlapping spheres in [0, L)^3."""
    cells = _Cells(L, a)
    out = np.empty((N, 3))
    n = 0
    tries = 0
    while n < N:
        p = rng.uniform(0.0, L, size=3)
        tries += 1
        if tries > max_tries * N:
            raise RuntimeError("random sequential addition did not converge")
        if cells.overlaps(p):
            continue
        cells.add(p)
        out[n] = p
        n += 1
    return out


def rod_positions(n_rods, per_rod, L, a, rng, max_tries=200):
    """Rods of ``per_rod`` touching spheres (spacing 2a) with uniform centres
    and uniform orientations, every sphere of every rod in x in [0, L/2)."""
    cells = _Cells(L, a)
    half = 0.5 * (per_rod - 1) * 2.0 * a
    offs = (np.arange(per_rod) - 0.5 * (per_rod - 1)) * 2.0 * a
    out = np.empty((n_rods * per_rod, 3))
    n = 0
    tries = 0
    while n < n_rods:
        tries += 1
        if tries > max_tries * n_rods:
            raise RuntimeError("rod placement did not converge")
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        ext = half * abs(u[0])
        cx = rng.uniform(ext, 0.5 * L - ext)
        cy, cz = rng.uniform(0.0, L, size=2)
        pts = np.array([cx, cy, cz])[None, :] + offs[:, None] * u[None, :]
        pts[:, 1:] = np.mod(pts[:, 1:], L)
        if any(cells.overlaps(p) for p in pts):
            continue
        for p in pts:
            cells.add(p)
        out[n * per_rod:(n + 1) * per_rod] = pts
        n += 1
    return out


def rod_monolayer(n_rods, per_rod, Lxy, z0, a, rng):
    """A planar suspension of rods (the setting of the paper's rod runs, Sec.
    6.1): rod centres on a square lattice of the [0, Lxy)^2 plane at height
    z0, each rod turned by a uniform angle within the plane.  A rod is
    ``per_rod`` (even) spheres stacked as doublets: per_rod / 2 stations
    along the axis, spacing a sqrt(2), each holding two spheres offset by
    +-a/sqrt(2), the doublets alternating between the in-plane normal and z
    (length (per_rod/2 - 1) a sqrt(2) + 2a: 16.1a for 22 spheres)."""
    side = int(math.ceil(math.sqrt(n_rods)))
    s = Lxy / side
    ns = per_rod // 2
    length = (ns - 1) * a * math.sqrt(2.0) + 2.0 * a
    if s <= length:
        raise ValueError("rods too long for the lattice spacing")
    ax = (np.arange(ns) - 0.5 * (ns - 1)) * a * math.sqrt(2.0)
    h = a / math.sqrt(2.0)
    out = np.empty((n_rods * per_rod, 3))
    for r in range(n_rods):
        th = rng.uniform(0.0, 2.0 * math.pi)
        c = np.array([(r % side + 0.5) * s, (r // side + 0.5) * s, z0])
        u = np.array([math.cos(th), math.sin(th), 0.0])
        nrm = np.array([-math.sin(th), math.cos(th), 0.0])
        ez = np.array([0.0, 0.0, 1.0])
        pts = []
        for i in range(ns):
            d = nrm if i % 2 == 0 else ez
            pts.append(c + ax[i] * u + h * d)
            pts.append(c + ax[i] * u - h * d)
        out[r * per_rod:(r + 1) * per_rod] = np.array(pts)
    return out


def filament_array(n_fil, per_fil, Lxy, dl, a, rng):
    """Filaments tethered on a square lattice of the plane z = 0 (the setting
    of the paper's filament runs, Sec. 6.2): ``per_fil`` segments spaced dl
    along a direction tilted from the z axis by up to 30 degrees."""
    side = int(math.ceil(math.sqrt(n_fil)))
    s = Lxy / side
    out = np.empty((n_fil * per_fil, 3))
    for f in range(n_fil):
        th = rng.uniform(0.0, math.pi / 6.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        u = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        base = np.array([(f % side + 0.5) * s, (f // side + 0.5) * s, a])
        out[f * per_fil:(f + 1) * per_fil] = base[None, :] + (np.arange(per_fil) * dl)[:, None] * u[None, :]
    return out


def box_for_fraction(N, a, phi):
    """Side L of the cube holding N spheres of radius a at volume fraction phi."""
    return (N * 4.0 * math.pi * a ** 3 / 3.0 / phi) ** (1.0 / 3.0)


def workload(index, N=None):
    """Inputs and run parameters of workload ``index`` (see the module doc).

    ``N`` overrides the particle count of workloads 1-2 (keeping the volume
    fraction), for scaled-down checks.  Returns a dict with keys
    name, N, L, a, eta, grid, Sigma, M_G, R_c, Y, F, T.
    """
    rng = rng_for(index)
    a, eta = 1.0, 1.0
    sigma = a / math.sqrt(math.pi)
    if index == 0:
        N = 64 if N is None else N
        L, grid, MG = 40.0, 32, 12
        Sigma, R_c = 2.0 * sigma, C1_RCUT
        Y = rsa_positions(N, L, a, rng)
        F = rng.normal(size=(N, 3))
        F -= F.mean(axis=0)
        T = rng.normal(size=(N, 3))
        name = "small N=64 L=40 grid32 FP64 parity"
    elif index in (1, 2):
        phi, grid = (0.01, 128) if index == 1 else (0.10, 256)
        N0 = 10_000 if index == 1 else 100_000
        N = N0 if N is None else N
        L = box_for_fraction(N0, a, phi)
        if N != N0:
            L = box_for_fraction(N, a, phi)
        Sigma = L / grid
        MG, R_c = 10, 5.5 * Sigma
        Y = rsa_positions(N, L, a, rng)
        F = rng.normal(size=(N, 3))
        T = rng.normal(size=(N, 3))
        name = ("dilute" if index == 1 else "dense") + f" N={N} phi={phi} grid{grid}"
    elif index == 3:
        n_rods = 2000 if N is None else max(N // 30, 1)
        L, grid = 600.0, 192
        Sigma = L / grid
        MG, R_c = 10, 5.5 * Sigma
        Y = rod_positions(n_rods, 30, L, a, rng)
        N = len(Y)
        F = np.zeros((N, 3))
        F[:, 0] = 1.0
        F += rng.normal(scale=0.1, size=(N, 3))
        T = np.zeros((N, 3))
        name = f"rods {n_rods}x30 L=600 grid192"
    else:
        raise ValueError(f"no workload {index}")
    return dict(name=name, N=N, L=L, a=a, eta=eta, grid=grid, Sigma=Sigma, M_G=MG,
                R_c=R_c, Y=Y, F=F, T=T)


def smooth_grid(n):
    """Smallest even 2^p 3^q >= n."""
    best = None
    p2 = 2
    while p2 < 4 * max(n, 2):
        v = p2
        while True:
            if v >= n and (best is None or v < best):
                best = v
            if v >= n:
                break
            v *= 3
        p2 *= 2
    return best


# Optimal Sigma/sigma of the paper's Table 3 (epsilon = 1e-4, a/L = 1/400).
_T3_PHI = np.array([0.0005, 0.002, 0.008, 0.032, 0.128])
_T3_RATIO = np.array([5.9, 5.1, 3.4, 1.8, 1.4])


def serving_stream(n_requests=512, seed_offset=4, n_lo=1_000, n_hi=200_000, rate=None):
    """Mixed-size request stream: N log-uniform in [n_lo, n_hi], volume
    fraction uniform in [1 %, 15 %], Sigma/sigma from Table 3 interpolated in
    log(phi) (1.4 above 12.8 %), grid the smallest even 2^p 3^q >= 1.5 L / Sigma,
    M_G = 16, R_c = 5.5 Sigma; Poisson arrival offsets (seconds) at ``rate``
    requests/s when given.  Positions are drawn lazily by ``request_inputs``."""
    rng = rng_for(seed_offset)
    a = 1.0
    sigma = a / math.sqrt(math.pi)
    reqs = []
    t = 0.0
    for i in range(n_requests):
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        phi = rng.uniform(0.01, 0.15)
        L = box_for_fraction(N, a, phi)
        ratio = float(np.interp(math.log(phi), np.log(_T3_PHI), _T3_RATIO))
        Sigma = ratio * sigma
        grid = smooth_grid(int(math.ceil(1.5 * L / Sigma)))
        gap = rng.exponential(1.0 / rate) if rate else 0.0
        t += gap
        reqs.append(dict(id=i, N=N, phi=phi, L=L, a=a, eta=1.0, Sigma=Sigma, grid=grid,
                         M_G=16, R_c=5.5 * Sigma, arrival=t, seed=SEED_BASE + 1000 + i))
    return reqs


def lattice_positions(N, L, a, rng):
    """N non-overlapping centres in [0, L)^3: a random subset of the sites of a
    cubic lattice with spacing s = L / ceil(N^(1/3)), each displaced uniformly
    by at most (s - 2a)/2 per axis (fast; used for the request stream, where
    sequential addition of millions of spheres would dominate the run)."""
    n = int(math.ceil(N ** (1.0 / 3.0) - 1e-9))
    s = L / n
    if s <= 2.0 * a:
        raise ValueError("volume fraction too high for the jittered lattice")
    sites = rng.choice(n ** 3, size=N, replace=False)
    ijk = np.stack([sites % n, (sites // n) % n, sites // (n * n)], axis=1).astype(np.float64)
    jit = rng.uniform(-0.5, 0.5, size=(N, 3)) * (s - 2.0 * a)
    return np.mod((ijk + 0.5) * s + jit, L)


def request_inputs(req):
    """Positions (non-overlapping jittered lattice), F and T ~ N(0, 1) of one request."""
    rng = np.random.default_rng(req["seed"])
    Y = lattice_positions(req["N"], req["L"], req["a"], rng)
    F = rng.normal(size=(req["N"], 3))
    T = rng.normal(size=(req["N"], 3))
    return Y, F, T
