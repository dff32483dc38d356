"""Seeded synthetic initial fields, shared by the GPU tests, the benchmark and
the oracle's tests.

This module holds no step of the lattice Boltzmann scheme: it only draws
numbers and lays out initial density and velocity fields.  The coexistence
densities it interpolates between are passed in by the caller.

Shapes follow the paper's workloads:

* static drop (Sec. 5.3, Eq. 41): tanh profile of width W around a circle of
  radius r0 centred in the domain;
* flat slab (Sec. 5.1): liquid in the middle half of the domain in y;
* drop splashing on a film (Sec. 5.5): a film along the bottom wall and a
  falling drop above it.

Geometry conventions: node (x, y) sits at integer coordinates, the domain
centre is (nx/2, ny/2), distances are plain Euclidean (no minimum image).
Noise is relative, rho <- rho (1 + amp xi), xi uniform in [-1, 1), drawn from
SplitMix64 (Steele, Lea and Flood, 2014) as a counter-based generator:
value number n of stream `seed` is mix(seed + (n + 1) * 0x9E3779B97F4A7C15).
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n):
    """First n outputs of SplitMix64 for stream `seed` (uint64 array)."""
    with np.errstate(over="ignore"):
        idx = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed) + idx * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed, n):
    """Doubles in [0, 1): the top 53 bits of each SplitMix64 output."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _tanh_blend(rho_g, rho_l, d, width):
    """(rho_g + rho_l)/2 + (rho_g - rho_l)/2 tanh(2 d / W): gas for d >> 0,
    liquid for d << 0 (d = signed distance to the interface)."""
    return 0.5 * (rho_g + rho_l) + 0.5 * (rho_g - rho_l) * np.tanh(2.0 * d / width)


def _coords(nx, ny):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    return x, y


def add_noise(rho, seed, amp):
    if amp == 0.0:
        return rho
    xi = 2.0 * uniform01(seed, rho.size).reshape(rho.shape) - 1.0
    return rho * (1.0 + amp * xi)


def droplet(nx, ny, rho_g, rho_l, radius, width, *, center=None, seed=0, noise=0.0):
    """Static drop: rho0 (ny, nx), ux0, uy0 (zeros)."""
    x, y = _coords(nx, ny)
    cx, cy = (nx / 2.0, ny / 2.0) if center is None else center
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    rho = add_noise(_tanh_blend(rho_g, rho_l, r - radius, width), seed, noise)
    z = np.zeros_like(rho)
    return np.ascontiguousarray(rho), z, z.copy()


def slab(nx, ny, rho_g, rho_l, width, *, seed=0, noise=0.0):
    """Flat liquid slab for ny/4 <= y < 3 ny/4 with two planar interfaces."""
    x, y = _coords(nx, ny)
    d = np.abs(y - (ny / 2.0 - 0.5)) - ny / 4.0
    rho = add_noise(_tanh_blend(rho_g, rho_l, d, width), seed, noise)
    z = np.zeros_like(rho)
    return np.ascontiguousarray(rho), z, z.copy()


def splash(nx, ny, rho_g, rho_l, radius, width, *, film=40, drop_center=None, drop_uy=-0.05,
           frame_ux=0.0, smooth_velocity=False):
    """Drop falling onto a liquid film lying on the bottom wall: film for
    y < `film`, drop of radius `radius` centred at `drop_center` (default
    (nx/2, film + radius + 10)).  The drop moves with (0, drop_uy) where its
    liquid fraction exceeds one half, or (smooth_velocity) with drop_uy times
    its liquid fraction, so that the velocity follows the tanh profile of the
    density; `frame_ux` is added to every node (reference frame moving to the
    right)."""
    x, y = _coords(nx, ny)
    cx, cy = (nx / 2.0, film + radius + 10.0) if drop_center is None else drop_center
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    phi_drop = 0.5 * (1.0 - np.tanh(2.0 * (r - radius) / width))
    phi_film = 0.5 * (1.0 - np.tanh(2.0 * (y - (film - 0.5)) / width))
    phi = np.maximum(phi_drop, phi_film)
    rho = rho_g + (rho_l - rho_g) * phi
    ux = np.full_like(rho, frame_ux)
    uy = drop_uy * phi_drop if smooth_velocity else np.where(phi_drop > 0.5, drop_uy, 0.0)
    return np.ascontiguousarray(rho), ux, np.ascontiguousarray(uy)


SWEEP_SIZES = (64, 128, 256, 512)


def sweep_members(seed, count, *, sizes=SWEEP_SIZES, t_lo=0.35, t_hi=0.95, r_lo=0.15,
                  r_hi=0.35):
    """Members of a batched sweep: square periodic meshes of side drawn
    uniformly from `sizes`, the first half flat slabs and the second half
    static drops of radius r N with r uniform in [r_lo, r_hi), each at a
    reduced temperature uniform in [t_lo, t_hi).  Returns a list of dicts
    {"kind", "n", "T_r", "radius"} (radius None for slabs).  Three draws per
    member from stream `seed`: size, temperature, radius."""
    u = uniform01(seed, 3 * count).reshape(count, 3)
    out = []
    for i in range(count):
        n = sizes[min(int(u[i, 0] * len(sizes)), len(sizes) - 1)]
        T_r = t_lo + (t_hi - t_lo) * float(u[i, 1])
        drop = i >= count // 2
        radius = (r_lo + (r_hi - r_lo) * float(u[i, 2])) * n if drop else None
        out.append({"kind": "drop" if drop else "slab", "n": n, "T_r": T_r, "radius": radius})
    return out


def warmstart_members(seed, count, *, t_lo, t_hi, r_lo, r_hi, k_lo, k_hi):
    """Static drops for the learned warm start: reduced temperature, radius
    fraction of the mesh side and mesh coefficient k, each uniform in its
    range; three draws per member from stream `seed`.  Returns a list of
    dicts {"T_r", "r_frac", "k"}."""
    u = uniform01(seed, 3 * count).reshape(count, 3)
    return [{"T_r": t_lo + (t_hi - t_lo) * float(a), "r_frac": r_lo + (r_hi - r_lo) * float(b),
             "k": k_lo + (k_hi - k_lo) * float(c)} for a, b, c in u]


def network_init(seed, n_in=7, n_hid=128, n_out=3):
    """Initial parameters of the n_in-n_hid-n_hid-n_out network in the flat
    order W1, b1, W2, b2, W3, b3: weights uniform in
    +-sqrt(6 / (fan_in + fan_out)) (Glorot and Bengio, 2010), biases zero;
    float32."""
    shapes = [(n_hid, n_in), (n_hid,), (n_hid, n_hid), (n_hid,), (n_out, n_hid), (n_out,)]
    total = sum(int(np.prod(s)) for s in shapes)
    u = 2.0 * uniform01(seed, total) - 1.0
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        if len(s) == 2:
            out.append(u[o:o + n] * np.sqrt(6.0 / (s[0] + s[1])))
        else:
            out.append(np.zeros(n))
        o += n
    return np.concatenate(out).astype(np.float32)


def minibatch_order(seed, nsamples, batch, iters):
    """iters * batch sample indices drawn uniformly (with replacement) from
    [0, nsamples), int32."""
    u = uniform01(seed, batch * iters)
    return np.minimum((u * nsamples).astype(np.int64), nsamples - 1).astype(np.int32)
