"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the lattice Boltzmann method: it only
draws random numbers and places particles.  Both the GPU library and the CPU
oracle receive what it produces as plain arrays.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the state advances by the
golden-ratio increment and each output is the state passed through the
variant-13 finaliser of MurmurHash3.  A uniform double in [0, 1) is the top
53 bits of an output times 2^-53.

Particle seeding is random sequential addition: candidate centres are drawn
uniformly (x first, then y) and accepted when the surface gap to every
accepted particle is at least `min_gap` (minimum image along the periodic x
axis) and the disk keeps the same clearance `min_gap` from both flat walls,
which sit halfway between nodes at y = -1/2 and y = ny - 1/2.  After 1000 * n attempts
without completing the set, seeding fails.
"""
import math

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


class SplitMix64:
    def __init__(self, seed):
        self.state = int(seed) & MASK64

    def next_u64(self):
        self.state = (self.state + GOLDEN_GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self):
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


class SeedingError(RuntimeError):
    pass


def rsa_particles(nx, ny, n, diameter, min_gap=1.0, seed=1):
    """Return an (n, 7) array of rows (x, y, r, ux, uy, theta, omega), all at rest.

    The acceptance test is evaluated exactly as written (binary64, no fused
    operations), so any implementation of the same steps gives bit-identical
    centres.
    """
    r = 0.5 * diameter
    ylo = (-0.5 + min_gap) + r
    yhi = ((ny - 0.5) - min_gap) - r
    if n < 0 or not (r > 0.0):
        raise ValueError("need n >= 0 and diameter > 0")
    if n > 0 and yhi < ylo:
        raise SeedingError("channel too narrow for the particles")
    rng = SplitMix64(seed)
    cell = 2.0 * r + max(min_gap, 0.0)
    ncx = max(1, int(nx // cell))
    ncy = max(1, int(ny // cell))
    grid = {}
    xs, ys = [], []
    half = 0.5 * nx
    attempts = 0
    while len(xs) < n:
        if attempts >= 1000 * n:
            raise SeedingError(f"placed {len(xs)} of {n} particles in {attempts} attempts")
        attempts += 1
        x = rng.uniform() * nx
        y = ylo + rng.uniform() * (yhi - ylo)
        cx = min(int(x / nx * ncx), ncx - 1)
        cy = min(max(int((y + 0.5) / ny * ncy), 0), ncy - 1)
        ok = True
        for dcy in (-1, 0, 1):
            yy = cy + dcy
            if yy < 0 or yy >= ncy:
                continue
            for dcx in (-1, 0, 1):
                for q in grid.get(((cx + dcx) % ncx, yy), ()):
                    dx = x - xs[q]
                    if dx > half:
                        dx = dx - nx
                    elif dx < -half:
                        dx = dx + nx
                    dy = y - ys[q]
                    gap = (math.sqrt(dx * dx + dy * dy) - r) - r
                    if gap < min_gap:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            grid.setdefault((cx, cy), []).append(len(xs))
            xs.append(x)
            ys.append(y)
    out = np.zeros((n, 7))
    out[:, 0] = xs
    out[:, 1] = ys
    out[:, 2] = r
    return out


def grid_particles(nx, ny, rows, cols, diameter, spacing):
    """Particles at rest on a regular grid hanging from the top of a closed
    cavity (walls at x = -1/2, nx - 1/2 and y = -1/2, ny - 1/2): `cols` per
    line centred across the width at `spacing` apart, `rows` lines from the
    top down, the top line one half spacing below the top wall.  Row-major
    from the top left."""
    width = cols * spacing
    if width > nx or rows * spacing > ny or diameter > spacing:
        raise ValueError("grid does not fit the cavity")
    x0 = -0.5 + 0.5 * (nx - width) + 0.5 * spacing
    y0 = (ny - 0.5) - 0.5 * spacing
    out = np.zeros((rows * cols, 7))
    for j in range(rows):
        for i in range(cols):
            out[j * cols + i, 0] = x0 + i * spacing
            out[j * cols + i, 1] = y0 - j * spacing
    out[:, 2] = 0.5 * diameter
    return out


def ring_cluster_ellipses(centre, counts, ring_spacing, a, b, theta=0.0):
    """Ellipses at rest in a circular cluster: one at `centre`, then ring k
    (k = 1, 2, ...) of counts[k - 1] particles at radius k * ring_spacing,
    evenly spaced in angle starting from +x, all with semi-axes (a, b) and
    body angle `theta`.  Rows of (x, y, a, b, ux, uy, theta, omega)."""
    cx, cy = centre
    rows = [[cx, cy, a, b, 0.0, 0.0, theta, 0.0]]
    for k, m in enumerate(counts, start=1):
        R = k * ring_spacing
        for j in range(m):
            phi = 2.0 * math.pi * j / m
            rows.append([cx + R * math.cos(phi), cy + R * math.sin(phi), a, b, 0.0, 0.0, theta, 0.0])
    return np.array(rows)


def workload_particles(w):
    """Initial particle rows of a workload description: `layout` "grid"
    (rows x cols at `spacing`), "rings" (an elliptical-particle cluster:
    rows of 8 values) or, by default, random sequential addition with its
    gap and seed."""
    if w.get("layout") == "grid":
        return grid_particles(w["nx"], w["ny"], w["rows"], w["cols"], w["d"], w["spacing"])
    if w.get("layout") == "rings":
        return ring_cluster_ellipses(w["centre"], w["rings"], w["ring_spacing"], 0.5 * w["d"],
                                     0.5 * w["d_minor"], w.get("theta", 0.0))
    return rsa_particles(w["nx"], w["ny"], w["n"], w["d"], w["gap"], w["seed"])


def smooth_fields(nx, ny, seed, amp_u=0.02, amp_T=0.5, modes=3, rho0=1.0):
    """Smooth random macroscopic fields (rho, ux, uy, T), each (ny, nx).

    A few Fourier modes, periodic in x and vanishing velocity at the walls, with
    SplitMix64-drawn amplitudes and phases.  They serve as initial conditions
    for parity runs of the lattice without particles.
    """
    rng = SplitMix64(seed)
    x = np.arange(nx)[None, :] + 0.0
    y = np.arange(ny)[:, None] + 0.0
    H = float(ny)
    wall = np.sin(np.pi * (y + 0.5) / H)
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    T = np.zeros((ny, nx))
    rho = np.full((ny, nx), rho0)
    for m in range(1, modes + 1):
        a = [rng.uniform() - 0.5 for _ in range(6)]
        ph = [2 * np.pi * rng.uniform() for _ in range(4)]
        kx = 2 * np.pi * m / nx
        ky = np.pi * m / H
        ux += amp_u * a[0] * wall * np.cos(kx * x + ph[0]) * np.cos(ky * (y + 0.5))
        uy += amp_u * a[1] * wall * np.sin(kx * x + ph[1]) * np.sin(ky * (y + 0.5))
        T += amp_T * a[2] * np.cos(kx * x + ph[2]) * np.sin(ky * (y + 0.5))
        rho += 0.01 * a[3] * np.cos(kx * x + ph[3]) * np.cos(ky * y)
    return rho, ux, uy, T


def random_state(n, seed, lo=0.0, hi=1.0):
    """n uniform doubles in [lo, hi) from SplitMix64."""
    rng = SplitMix64(seed)
    return np.array([lo + (hi - lo) * rng.uniform() for _ in range(n)])


def _uniform_int(rng, lo, hi):
    """Integer uniform on [lo, hi] from one draw."""
    return lo + min(int(rng.uniform() * (hi - lo + 1)), hi - lo)


def serving_requests(n=256, seed=4, L_range=(128, 1024), np_range=(5, 400), d_range=(8, 24),
                     Ra_range=(1e5, 1e8), steps_range=(500, 5000), max_fill=0.2):
    """A seeded mix of independent simulation requests for the serving form.

    Per request, in draw order: edge L = round(exp(U[ln L_lo, ln L_hi])); aspect
    A = 1 if the next draw is < 1/2 else 2, with nx = L, ny = A L; diameter d
    uniform integer in d_range; particle count uniform integer in np_range,
    then lowered to the largest count whose disks cover at most max_fill of the
    lattice; Ra = exp(U[ln Ra_lo, ln Ra_hi]); step count uniform integer in
    steps_range.  Each request also carries the seed of its particle placement
    (seed * 100003 + index).
    """
    rng = SplitMix64(seed)
    out = []
    for i in range(n):
        L = int(round(math.exp(math.log(L_range[0]) + rng.uniform() *
                               (math.log(L_range[1]) - math.log(L_range[0])))))
        A = 1 if rng.uniform() < 0.5 else 2
        d = float(_uniform_int(rng, int(d_range[0]), int(d_range[1])))
        n_p = _uniform_int(rng, np_range[0], np_range[1])
        n_fill = int(max_fill * L * A * L / (math.pi * d * d / 4.0))
        n_p = max(0, min(n_p, n_fill))
        Ra = math.exp(math.log(Ra_range[0]) + rng.uniform() * (math.log(Ra_range[1]) - math.log(Ra_range[0])))
        steps = _uniform_int(rng, steps_range[0], steps_range[1])
        out.append(dict(rid=i, nx=L, ny=A * L, d=d, n=n_p, Ra=Ra, steps=steps,
                        seed=seed * 100003 + i))
    return out


def poisson_arrivals(n, rate, seed):
    """Arrival times (seconds, from 0) of a Poisson process of the given rate:
    cumulative sums of exponential gaps -ln(1 - U) / rate."""
    rng = SplitMix64(seed)
    t, out = 0.0, []
    for _ in range(n):
        t += -math.log(1.0 - rng.uniform()) / rate
        out.append(t)
    return np.array(out)
