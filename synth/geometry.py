"""Seeded periodic voxel geometries and random fields.

Conventions: a mask is a uint8 array of shape (N, N, N) indexed [k][j][i]
(x fastest), 1 = fluid, 0 = solid, periodic in all three directions.  The flat
index of voxel (i, j, k) is i + N*(j + N*k).

The paper's own CT images and 2D square packings are not available; these
generators stand in for them with the shapes, porosities and surface-to-volume
ratios of the paper's regime (porosity 4-42 %, surface-to-volume 14-74 %,
Tables of the 3D samples and of the 2D channel-width sweep).
"""

from __future__ import annotations

import numpy as np


def porosity(mask: np.ndarray) -> float:
    """Fluid fraction of a voxel mask."""
    return float(np.count_nonzero(mask)) / mask.size


def _ball_offsets(radius: float):
    """Integer offsets of a cube that contains every voxel a ball of this radius can touch."""
    R = int(np.ceil(radius)) + 1
    o = np.arange(-R, R + 1)
    oz, oy, ox = np.meshgrid(o, o, o, indexing="ij")
    return ox.ravel(), oy.ravel(), oz.ravel()


def _sphere_voxels(N: int, centres: np.ndarray, radius: float, offs):
    """Flat indices of voxels whose centres lie in the closed periodic balls.

    centres: (B, 3) array of (x, y, z) in voxel units.  Distances use the
    periodic minimum image.
    """
    ox, oy, oz = offs
    base = np.floor(centres).astype(np.int64)                     # (B,3)
    vi = base[:, 0:1] + ox[None, :]
    vj = base[:, 1:2] + oy[None, :]
    vk = base[:, 2:3] + oz[None, :]
    dx = vi + 0.5 - centres[:, 0:1]
    dy = vj + 0.5 - centres[:, 1:2]
    dz = vk + 0.5 - centres[:, 2:3]
    dx -= N * np.round(dx / N)
    dy -= N * np.round(dy / N)
    dz -= N * np.round(dz / N)
    inside = dx * dx + dy * dy + dz * dz <= radius * radius
    flat = (vi % N) + N * ((vj % N) + N * (vk % N))
    return flat, inside


def spheres(N: int, radius: float, target_porosity: float, seed: int,
            batch: int = 512) -> np.ndarray:
    """Overlapping solid spheres until the porosity first drops to the target.

    Centres are drawn one after another as rng.uniform(0, N, 3) from
    numpy.random.default_rng(seed) (drawing them in blocks gives the same
    stream).  A voxel is solid when its centre lies within the closed ball of
    the given radius under the periodic minimum-image distance.  Spheres are
    added until porosity <= target; the first crossing stops.
    """
    rng = np.random.default_rng(seed)
    n3 = N * N * N
    fluid = np.ones(n3, dtype=np.uint8)
    n_fluid = n3
    target_fluid = target_porosity * n3
    offs = _ball_offsets(radius)
    while n_fluid > target_fluid:
        centres = rng.uniform(0, N, (batch, 3))
        flat, inside = _sphere_voxels(N, centres, radius, offs)
        trial = fluid.copy()
        trial[flat[inside]] = 0
        n_trial = int(np.count_nonzero(trial))
        if n_trial > target_fluid:
            fluid, n_fluid = trial, n_trial
            continue
        # the crossing happens inside this block: replay it sphere by sphere
        for b in range(batch):
            idx = np.unique(flat[b][inside[b]])
            n_fluid -= int(np.count_nonzero(fluid[idx]))
            fluid[idx] = 0
            if n_fluid <= target_fluid:
                break
        break
    return fluid.reshape(N, N, N)


def grf(N: int, corr_len: float, target_porosity: float, seed: int,
        kernel_std: float | None = None) -> np.ndarray:
    """Thresholded Gaussian random field, fluid = 1.

    White noise rng.standard_normal((N, N, N)) is smoothed by periodic
    convolution with a Gaussian kernel of standard deviation corr_len/sqrt(2)
    voxels (so the field covariance is exp(-r^2 / (2 corr_len^2))), then the
    top target_porosity fraction of voxels (ties broken by flat index) is fluid.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N, N))
    s = corr_len / np.sqrt(2.0) if kernel_std is None else kernel_std
    kz = 2 * np.pi * np.fft.fftfreq(N)
    kx = 2 * np.pi * np.fft.rfftfreq(N)
    filt = np.exp(-0.5 * s * s * (kz[:, None, None] ** 2 + kz[None, :, None] ** 2
                                  + kx[None, None, :] ** 2))
    field = np.fft.irfftn(np.fft.rfftn(w) * filt, s=(N, N, N), axes=(0, 1, 2)).ravel()
    del w
    n_fluid = int(round(target_porosity * field.size))
    order = np.argsort(-field, kind="stable")
    fluid = np.zeros(field.size, dtype=np.uint8)
    fluid[order[:n_fluid]] = 1
    return fluid.reshape(N, N, N)


def slits(N: int, widths, wall: int = 2, axis: int = 1) -> np.ndarray:
    """Stack of plane channels separated by solid walls normal to `axis`.

    Starting at index 0 along `axis`: `wall` solid rows, then a channel of
    widths[0] fluid rows, `wall` solid rows, widths[1] fluid rows, ...; the
    width list repeats until N rows are filled (truncated at N; a trailing
    partial channel is closed by the wall at index 0 through periodicity).
    With a single width W this is "row mod (W + wall) < wall is solid".
    axis: 0 = walls normal to x, 1 = normal to y, 2 = normal to z.
    """
    if np.isscalar(widths):
        widths = [int(widths)]
    rows = []
    n = 0
    while len(rows) < N:
        rows.extend([0] * wall)
        rows.extend([1] * int(widths[n % len(widths)]))
        n += 1
    prof = np.array(rows[:N], dtype=np.uint8)
    shape = [1, 1, 1]
    shape[2 - axis] = N                      # array order is [k][j][i]
    return np.broadcast_to(prof.reshape(shape), (N, N, N)).copy()


def channel_widths(N: int, widths, wall: int = 2):
    """Fluid widths of the channels `slits` produces (the trailing one may be cut)."""
    if np.isscalar(widths):
        widths = [int(widths)]
    out = []
    pos = 0
    n = 0
    while pos < N:
        pos += wall
        w = int(widths[n % len(widths)])
        if pos < N:
            out.append(min(w, N - pos))
        pos += w
        n += 1
    return out


def random_face_field(N: int, seed: int) -> np.ndarray:
    """Standard-normal face field, shape (3, N, N, N): component c is the velocity on
    the lower c-faces of every voxel."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, N, N, N))


def random_cell_field(N: int, seed: int) -> np.ndarray:
    """Standard-normal cell field, shape (N, N, N)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, N, N))
