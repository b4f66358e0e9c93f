"""Named synthetic workloads shaped like the paper's cases.

The paper's sample PSFs (wave-optics microscope PSFs, and an experimental
camera PSF) are not available, so each workload is a seeded Gaussian-envelope
array of the same shape class: patch rows x patch columns x cell rows x cell
columns x depths, float32.  The sigma of the envelope grows linearly with the
distance from the central depth, as PSF patterns widen away from focus.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Workload:
    name: str
    shape: tuple            # (ns, nt, nx, ny, nz)
    sig0: float             # envelope sigma at the central depth, px
    slope: float            # sigma growth per depth step, px
    zc: float               # central depth index (0-based)
    seed: int

    @property
    def elements(self) -> int:
        ns, nt, nx, ny, nz = self.shape
        return ns * nt * nx * ny * nz


# Nnum = 3, 15x15 px patches, 3 depths: small enough for the dense oracle.
TINY = Workload("tiny", (15, 15, 3, 3, 3), 0.8, 0.6, 1.0, 1)
# Microscope: Nnum = 15, 165x165 px patches (11 lenslets), 21 depths (~0.5 GB f32).
MICROSCOPE = Workload("microscope", (165, 165, 15, 15, 21), 1.0, 0.5, 10.0, 2)
# Camera: Nnum = 15, 345x345 px patches (23 lenslets), 51 depths (~5.5 GB f32).
CAMERA = Workload("camera", (345, 345, 15, 15, 51), 1.0, 0.4, 25.0, 3)


def batched_set(i: int) -> Workload:
    """Set i of the 16-set batch: Nnum cycles through 7, 11, 15, 19; the lenslet
    count L through the odd values 9..25; depth count nz = 9 + (13 i mod 33)."""
    nnum = (7, 11, 15, 19)[i % 4]
    lens = (9, 11, 13, 15, 17, 19, 21, 23, 25)[(5 * i + i // 4) % 9]
    nz = 9 + (13 * i) % 33
    patch = lens * nnum
    return Workload(f"batch{i}", (patch, patch, nnum, nnum, nz), 1.0, 0.4, (nz - 1) / 2.0, 1000 + i)


BATCHED_SETS = tuple(batched_set(i) for i in range(16))


def small_set(i: int) -> Workload:
    """Set i of the 64-set batch of small PSFs (a depth or lens sweep of a small
    system, where per-launch overhead is comparable with the work): Nnum cycles
    through 3, 5, 7; the lenslet count through 3, 5, 7; nz = 4 + (7 i mod 11)."""
    nnum = (3, 5, 7)[i % 3]
    lens = (3, 5, 7)[(i // 3 + i) % 3]
    nz = 4 + (7 * i) % 11
    patch = lens * nnum
    return Workload(f"small{i}", (patch, patch, nnum, nnum, nz), 0.8, 0.4, (nz - 1) / 2.0, 2000 + i)


SMALL_SETS = tuple(small_set(i) for i in range(64))


@dataclass(frozen=True)
class ProjectorWorkload:
    name: str
    psf: Workload           # PSF array used by the projector
    lenslets: int           # lenslets per image side
    g_seed: int             # seed of the volume g ~ U[0,1)

    @property
    def image(self) -> tuple:
        nx = self.psf.shape[2]
        return (self.lenslets * nx, self.lenslets * self.psf.shape[3])


# 40 x 40 lenslets of Nnum = 15 -> 600 x 600 px image, 21 depths, microscope PSF.
PROJECTOR = ProjectorWorkload("projector", MICROSCOPE, 40, 5)

# Table 1 shapes (patch side, cell rows, cell columns), all with 11 depths.
TABLE1_SHAPES = ((89, 11, 11), (177, 11, 11), (287, 11, 11), (507, 11, 11), (91, 15, 15),
                 (121, 15, 15), (211, 21, 21), (249, 31, 31), (311, 31, 31), (307, 51, 51),
                 (181, 95, 55))


def table1_workload(i: int) -> Workload:
    """Row i of Table 1 as a workload: the paper's array size with 11 depths,
    Gaussian envelope centred on the middle depth."""
    patch, nx, ny = TABLE1_SHAPES[i]
    return Workload(f"table1-{patch}-{nx}x{ny}", (patch, patch, nx, ny, 11), 1.0, 0.4, 5.0, 3000 + i)
