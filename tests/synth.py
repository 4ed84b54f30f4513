"""Seeded synthetic fields shaped like the paper's evaluation workloads.

The SDRBench fields of the paper's Table 1 are not available, so these stand
in for them: same shapes, comparable value structure.  This module holds no
compression arithmetic; it only draws inputs, and both the oracle and the HIP
path consume what it returns.  Everything is generated in float64 with numpy's
PCG64 and cast to float32 at the end.

Workloads (recipes):
  sine3d(64,64,64)      sum of 8 random 3-D sine modes, amplitude U(0.5,1),
                         wavelength U(8,64) cells, direction uniform on the
                         sphere, phase U(0,2pi); plus N(0,1e-3) noise.
  climate2d(1800,3600)  16 random 2-D modes; then one axis-aligned rectangle
                         covering 20% of the area set to exactly 0.
  hurricane3d(100,500,500)  12 3-D modes plus a vortex r*exp(-r^2/sigma^2)
                         (sigma = 40 cells), r = distance in (x,y) from the
                         slanted axis (x0 + 0.3 z, y0 + 0.2 z).
  lognormal3d(512)      exp(G), G a Gaussian random field with power spectrum
                         k^-3 (k >= 1), normalised to mean 0 and sigma 1.5.
  batch_fields(n)       mixed-rank fields, sizes log-uniform 16 KiB-64 MiB,
                         aspect ratios log-uniform in [1/4, 4], values as the
                         sine workload in the field's rank.
"""
import numpy as np


def _grid(shape):
    return np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij", sparse=True)


def _modes(shape, n_modes, rng, lam=(8.0, 64.0)):
    """Sum of random plane-wave sine modes over a grid of any rank."""
    rank = len(shape)
    coords = _grid(shape)
    f = np.zeros(shape, dtype=np.float64)
    for _ in range(n_modes):
        amp = rng.uniform(0.5, 1.0)
        wl = rng.uniform(*lam)
        k = rng.normal(size=rank)
        k /= np.linalg.norm(k)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        arg = ph
        for d in range(rank):
            arg = arg + (2.0 * np.pi / wl) * k[d] * coords[d]
        f += amp * np.sin(arg)
    return f


def sine_field(shape, seed, noise=1e-3):
    rng = np.random.default_rng(seed)
    f = _modes(tuple(shape), 8, rng)
    if noise:
        f += rng.normal(0.0, noise, size=tuple(shape))
    return f.astype(np.float32)


def sine_field_device(shape, seed, device, noise=1e-3):
    """The sine workload generated on a torch device (for benchmarks that need
    gigabytes of fields quickly): the same seeded draws as sine_field for the
    mode parameters, the sum computed in float32 on the device and torch's
    own seeded normal noise, so values follow the same recipe but are not
    bit-identical to sine_field's."""
    import torch

    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in shape)
    rank = len(shape)
    coords = [torch.arange(n, dtype=torch.float32, device=device).view(*[n if d == i else 1 for d in range(rank)])
              for i, n in enumerate(shape)]
    f = torch.zeros(shape, dtype=torch.float32, device=device)
    for _ in range(8):
        amp = rng.uniform(0.5, 1.0)
        wl = rng.uniform(8.0, 64.0)
        k = rng.normal(size=rank)
        k /= np.linalg.norm(k)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        arg = torch.full((1,) * rank, float(ph), dtype=torch.float32, device=device)
        for d in range(rank):
            arg = arg + float(2.0 * np.pi / wl * k[d]) * coords[d]
        f += float(amp) * torch.sin(arg)
    if noise:
        g = torch.Generator(device=device)
        g.manual_seed(int(seed))
        f += noise * torch.randn(shape, generator=g, device=device, dtype=torch.float32)
    return f.contiguous()


def sine3d(seed=0, shape=(64, 64, 64)):
    return sine_field(shape, seed)


def climate2d(seed=100, shape=(1800, 3600)):
    rng = np.random.default_rng(seed)
    f = _modes(tuple(shape), 16, rng)
    ny, nx = shape
    # axis-aligned rectangle of 20% of the area, aspect drawn at random
    frac = 0.2
    ay = rng.uniform(0.3, 0.7)
    h = int(round(ny * ay))
    w = int(round(frac * ny * nx / max(h, 1)))
    w = min(w, nx)
    y0 = int(rng.integers(0, ny - h + 1))
    x0 = int(rng.integers(0, nx - w + 1))
    f[y0:y0 + h, x0:x0 + w] = 0.0
    return f.astype(np.float32)


def hurricane3d(seed=200, shape=(100, 500, 500), sigma=40.0):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    f = np.empty(shape, dtype=np.float32)
    modes = []
    for _ in range(12):
        amp = rng.uniform(0.5, 1.0)
        wl = rng.uniform(8.0, 64.0)
        k = rng.normal(size=3)
        k /= np.linalg.norm(k)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        modes.append((amp, wl, k, ph))
    x0 = rng.uniform(0.3, 0.7) * nx
    y0 = rng.uniform(0.3, 0.7) * ny
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    for z in range(nz):  # plane by plane keeps the float64 footprint small
        plane = np.zeros((ny, nx), dtype=np.float64)
        for amp, wl, k, ph in modes:
            plane += amp * np.sin(ph + (2.0 * np.pi / wl) * (k[0] * z + k[1] * y + k[2] * x))
        r = np.sqrt((x - (x0 + 0.3 * z)) ** 2 + (y - (y0 + 0.2 * z)) ** 2)
        plane += r * np.exp(-(r * r) / (sigma * sigma))
        f[z] = plane.astype(np.float32)
    return f


def lognormal3d(seed=300, n=512, sigma=1.5):
    rng = np.random.default_rng(seed)
    try:
        import scipy.fft as sfft

        kw = dict(workers=-1)
        rfftn, irfftn = sfft.rfftn, sfft.irfftn
    except Exception:  # pragma: no cover - scipy is in the image
        kw = {}
        rfftn, irfftn = np.fft.rfftn, np.fft.irfftn
    w = rng.standard_normal(size=(n, n, n))
    W = rfftn(w, **kw)
    del w
    kz = (np.fft.fftfreq(n) * n)[:, None, None]
    ky = (np.fft.fftfreq(n) * n)[None, :, None]
    kx = (np.fft.rfftfreq(n) * n)[None, None, :]
    k2 = kz * kz + ky * ky + kx * kx
    amp = np.where(k2 >= 1.0, np.power(np.maximum(k2, 1.0), -0.75), 0.0)  # sqrt(k^-3)
    W *= amp
    del amp, k2
    g = irfftn(W, s=(n, n, n), axes=(0, 1, 2), **kw)
    del W
    g -= g.mean()
    g *= sigma / g.std()
    np.exp(g, out=g)
    return g.astype(np.float32)


def batch_shapes(n_fields=256, seed=3000, lo=16 << 10, hi=64 << 20):
    """Mixed-rank shapes with log-uniform byte sizes and aspect ratios."""
    shapes = []
    for i in range(n_fields):
        rng = np.random.default_rng(seed + i)
        rank = int(rng.integers(1, 4))
        nbytes = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        n = max(1, int(nbytes // 4))
        if rank == 1:
            shapes.append((n,))
            continue
        aspects = np.exp(rng.uniform(np.log(0.25), np.log(4.0), size=rank - 1))
        base = (n / np.prod(aspects)) ** (1.0 / rank)
        dims = [max(1, int(round(base)))] + [max(1, int(round(base * a))) for a in aspects]
        shapes.append(tuple(dims))
    return shapes


def batch_field(shape, seed):
    return sine_field(shape, seed)


def rel_eb_choice(seed):
    rng = np.random.default_rng(seed)
    return [1e-2, 1e-3, 1e-4][int(rng.integers(0, 3))]


def wide_field(shape, seed):
    """Values spanning several binades (smooth in log2), a few negative
    regions, and sparse zeros, fp32 denormals and values near 1e30: the
    workload of the point-wise relative mode."""
    rng = np.random.default_rng(seed)
    mag = np.exp(sine_field(shape, seed=seed).astype(np.float64) * 0.5)
    sign = np.where(sine_field(shape, seed=seed + 1) > 3.5, -1.0, 1.0)
    x = (mag * sign).astype(np.float32)
    flat = x.reshape(-1)
    # each special value costs up to 8 escaped deltas; a chunk holds at most 1024
    flat[::1009] = 0.0
    flat[7::2111] = np.float32(3e-42)
    flat[5::3001] = rng.standard_normal(flat[5::3001].size).astype(np.float32) * np.float32(1e30)
    return x


# ------------------------------------------------ seeded sweeps of shapes and values
BOX = {1: (32768,), 2: (32, 1024), 3: (16, 32, 64)}
MAX_VALUES = 400_000


def draw_shape(rng, rank):
    while True:
        shape = []
        for b in BOX[rank]:
            k = int(rng.integers(0, 4))
            base = b * int(rng.integers(1, 3)) if rank > 1 else b * int(rng.integers(1, 4))
            ext = {0: base, 1: base + 1, 2: max(1, base - 1), 3: int(rng.integers(1, 2 * b + 1))}[k]
            shape.append(ext)
        shape = tuple(shape)
        if np.prod(shape) <= MAX_VALUES:
            return shape


def draw_field(rng, shape, seed):
    kind = ["sine", "lognormal", "noise", "zeros_block", "signed_zero", "denormal", "patches"][int(rng.integers(0, 7))]
    if kind == "sine":
        x = sine_field(shape, seed=seed)
    elif kind == "lognormal":
        x = np.exp(rng.standard_normal(shape) * 1.5).astype(np.float32)
    elif kind == "noise":
        x = rng.standard_normal(shape).astype(np.float32)
    elif kind == "zeros_block":
        x = sine_field(shape, seed=seed)
        sl = tuple(slice(0, max(1, n // 2)) for n in shape)
        x[sl] = 0.0
    elif kind == "signed_zero":
        x = sine_field(shape, seed=seed)
        x[x < 0] = np.float32(-0.0)
    elif kind == "denormal":  # every 7th value a denormal, the range stays normal
        x = sine_field(shape, seed=seed)
        flat = x.reshape(-1)
        flat[::7] = (flat[::7] * np.float32(1e-39)).astype(np.float32)
    else:
        x = np.repeat(rng.standard_normal(max(1, x_len(shape) // 97 + 1)).astype(np.float32), 97)[:x_len(shape)]
        x = x.reshape(shape)
    return kind, np.ascontiguousarray(x, dtype=np.float32)


def x_len(shape):
    return int(np.prod(shape))




def spike_field(shape, count, rows, seed, amp=100000.0):
    """Zeros with `count` isolated spikes of height `amp` at even coordinates,
    their slowest coordinate in the half-open range `rows`.  Under an absolute
    bound of 0.5 (grid step 1) each spike's integer is `amp`, and its Lorenzo
    deltas (2^rank of them, +-amp, all inside the spike's chunk because chunk
    boxes have even extents) do not fit in 16 bits: `count * 2**rank` escaped
    codes whose positions the test controls."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in shape)
    cand = [np.arange(rows[0] + (rows[0] & 1), rows[1], 2)] + [np.arange(0, n, 2) for n in shape[1:]]
    total = int(np.prod([len(c) for c in cand]))
    if count > total:
        raise ValueError("too many spikes for the rows")
    pick = rng.choice(total, size=count, replace=False)
    idx = np.unravel_index(pick, [len(c) for c in cand])
    f = np.zeros(shape, dtype=np.float32)
    f[tuple(c[i] for c, i in zip(cand, idx))] = np.float32(amp)
    return f
