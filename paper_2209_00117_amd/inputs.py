"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the flooding method: it only draws initial seed
positions, sample pixels and the workload recipes, so that the HIP path and
the CPU oracle are fed identical inputs.  It imports neither of them.

Random numbers come from splitmix64 (Steele, Lea and Flood, OOPSLA 2014),
written here from its published definition: output n (n >= 0) of the stream
seeded with s is mix64(s + (n + 1) * 0x9E3779B97F4A7C15), with Stafford's
variant-13 mixer.  A draw r is mapped onto [0, m) by ((r >> 32) * m) >> 32.

The paper's workloads are uniform random seeds on square pixel grids with
uniform random moves (Sec. II, Sec. VI-A); the recipes below fix the sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the splitmix64 stream of `seed`."""
    n = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(seed) + (n + np.uint64(1)) * _GAMMA)


def bounded(r: np.ndarray, m) -> np.ndarray:
    """Maps 64-bit draws onto [0, m) (multiply-shift on the top 32 bits)."""
    with np.errstate(over="ignore"):
        return ((r >> np.uint64(32)) * np.uint64(m)) >> np.uint64(32)


def place_seeds(W: int, H: int, S: int, seed: int) -> np.ndarray:
    """S distinct uniform random pixels, as an (S, 2) int32 array of (x, y).

    Pair j of the stream is (x, y) = (bounded(out[2j], W), bounded(out[2j+1], H));
    pairs are taken in order and a pair whose pixel is already taken is
    skipped (rejection sampling), so seed i is the i-th distinct pixel drawn.
    """
    if not (1 <= S <= W * H):
        raise ValueError(f"need 1 <= S <= W*H, got S={S}, W*H={W * H}")
    taken = np.zeros(W * H, dtype=bool)
    out = np.empty((S, 2), dtype=np.int32)
    got = 0
    pair = 0
    while got < S:
        need = S - got
        chunk = int(min(max(4 * need, 4096), 1 << 22))
        r = splitmix64(seed, 2 * pair, 2 * chunk)
        x = bounded(r[0::2], W).astype(np.int64)
        y = bounded(r[1::2], H).astype(np.int64)
        pix = y * W + x
        _, first = np.unique(pix, return_index=True)      # first draw of each pixel in the chunk
        first.sort()
        first = first[~taken[pix[first]]]                  # drop pixels taken by earlier chunks
        first = first[:need]
        out[got:got + first.size, 0] = x[first]
        out[got:got + first.size, 1] = y[first]
        taken[pix[first]] = True
        got += first.size
        pair += chunk
    return out


def sample_pixels(W: int, H: int, n: int, seed: int = 7):
    """n uniform random pixels (repeats allowed) as (px, py) int32 arrays."""
    r = splitmix64(seed, 0, 2 * n)
    return (bounded(r[0::2], W).astype(np.int32), bounded(r[1::2], H).astype(np.int32))


# ---------------------------------------------------------------------------
# Workload recipes.
# ---------------------------------------------------------------------------
@dataclass
class SimSpec:
    width: int
    height: int
    num_seeds: int
    disp_lo: int
    disp_hi: int
    sim_seed: int
    steps: int

    def positions(self) -> np.ndarray:
        return place_seeds(self.width, self.height, self.num_seeds, self.sim_seed)

    @property
    def pixels(self) -> int:
        return self.width * self.height


@dataclass
class Workload:
    name: str
    sims: list = field(default_factory=list)
    sample_pixels: int = 0            # 0: similarity over every pixel


def small() -> Workload:
    """512 x 512, 256 seeds, 5 steps, moves in [-1, 1]."""
    return Workload("small 512x512 S=256 disp[-1,1]", [SimSpec(512, 512, 256, -1, 1, 1, 5)])


def single() -> Workload:
    """4096 x 4096, 65536 seeds, 100 steps, moves in [-2, 2]."""
    return Workload("single 4096x4096 S=65536 disp[-2,2]",
                    [SimSpec(4096, 4096, 65536, -2, 2, 1, 100)], sample_pixels=1 << 20)


def large() -> Workload:
    """8192 x 8192, 2^20 seeds, 50 steps, moves in [-4, 4]."""
    return Workload("large 8192x8192 S=2^20 disp[-4,4]",
                    [SimSpec(8192, 8192, 1 << 20, -4, 4, 1, 50)], sample_pixels=1 << 20)


def band() -> Workload:
    """One GPU's share of the 8192 x 8192 grid split into eight row bands:
    1024 rows plus 16 halo rows on each side (delta_1 = 16 at that density),
    with seeds at the same density (2^20 / 8 per 1024 rows), moves in
    [-4, 4]."""
    rows = 8192 // 8 + 2 * 16
    return Workload(f"band 8192x{rows} S={128 * rows} disp[-4,4] (one of 8 row bands of "
                    f"8192^2 with its 16-row halos)",
                    [SimSpec(8192, rows, 128 * rows, -4, 4, 1, 50)], sample_pixels=1 << 20)


def batched(n_sims: int = 64, steps: int = 20) -> Workload:
    """64 independent simulations; side drawn from {256, ..., 4096}, seed
    count uniform in [2^6, 2^16] (at most side^2), moves in [-1, 3]."""
    sides = (256, 512, 1024, 2048, 4096)
    r = splitmix64(1, 0, 2 * n_sims)
    sims = []
    for j in range(n_sims):
        side = sides[int(bounded(r[2 * j:2 * j + 1], 5)[0])]
        s = 64 + int(bounded(r[2 * j + 1:2 * j + 2], 65473)[0])
        sims.append(SimSpec(side, side, min(s, side * side), -1, 3, 1000 + j, steps))
    return Workload(f"batched {n_sims} sims sides 256..4096 S 2^6..2^16 disp[-1,3]", sims)


def serving(n_sims: int = 256) -> Workload:
    """256 resident simulations; side drawn from {512, ..., 4096}, seed count
    uniform in [2^8, 2^18] (at most side^2), moves in [-2, 2]."""
    sides = (512, 1024, 2048, 4096)
    r = splitmix64(3, 0, 2 * n_sims)
    sims = []
    for j in range(n_sims):
        side = sides[int(bounded(r[2 * j:2 * j + 1], 4)[0])]
        s = 256 + int(bounded(r[2 * j + 1:2 * j + 2], (1 << 18) - 256 + 1)[0])
        sims.append(SimSpec(side, side, min(s, side * side), -2, 2, 2000 + j, 0))
    return Workload(f"serving {n_sims} sims sides 512..4096 S 2^8..2^18 disp[-2,2]", sims)


def poisson_arrivals(rate_per_s: float, duration_s: float, n_sims: int, seed: int = 5):
    """Arrival times (s) and target simulations of a Poisson request stream:
    gaps are -ln(U)/rate with U a 53-bit uniform in (0, 1]."""
    times, targets = [], []
    t, n = 0.0, 0
    while True:
        r = splitmix64(seed, 2 * n, 2)
        u = (int(r[0]) >> 11) * (1.0 / (1 << 53))
        t += -math.log(1.0 - u) / rate_per_s
        if t >= duration_s:
            break
        times.append(t)
        targets.append(int(bounded(r[1:2], n_sims)[0]))
        n += 1
    return np.array(times), np.array(targets, dtype=np.int64)


WORKLOADS = {"small": small, "single": single, "large": large, "band": band,
             "batched": batched, "serving": serving}
