"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module only describes inputs: lattice sizes, physical parameters and
seeds.  It holds none of the method's arithmetic, so both the GPU library and
the CPU oracle can be driven from it without sharing any computation.

The parameter set follows the problem statement of Sec. III.A of the paper
(Lx x L lattice, periodic x, walls at z = +-L/2, imposed gradient grad_c0,
thermal energy kT, coupling G, relaxation times, rho_bar = 1, c_bar0 = 1/2).
"""
from __future__ import annotations

import dataclasses
from typing import List

# option flags (bit values; the GPU header and the oracle each define their own
# copies of the same numbers)
ASTAR = 1            # a_* correction of the footnote to Eq. (13)
WALL_UZ_FIX = 2      # U_z = 0 on the wall rows (Sec. III.A)
NOISE_LOC = 4        # local instead of reference densities in the noise
FORCE_LITERAL = 8    # first-order forcing without (1 - lambda_d/2) (tests only)
NO_GRAPH = 16        # execution only: no graph replay
SAMPLE_VELOCITY = 32 # also sample U_x, U_z for the velocity structure factors
TWO_STEP = 64        # execution only: pairs of steps in the two-step kernel
ONE_STEP = 128       # execution only: one step per launch
DEFAULT_FLAGS = ASTAR | WALL_UZ_FIX


@dataclasses.dataclass
class Replica:
    """One lattice: geometry, physics and its Philox seed."""
    Lx: int
    Lz: int
    rho0: float = 1.0
    grad_c0: float = 0.0
    kT: float = 0.0
    G: float = 0.0
    tau_d: float = 1.0
    tau_s: float = 1.0
    tau_e: float = 1.0
    tau_q: float = 1.0
    tau_eps: float = 1.0
    seed: int = 1

    @property
    def nodes(self) -> int:
        return self.Lx * self.Lz


def splitmix64(seed: int, n: int) -> List[int]:
    """The first n outputs of SplitMix64 (Steele, Lea, Flood 2014)."""
    mask = (1 << 64) - 1
    out = []
    x = seed & mask
    for _ in range(n):
        x = (x + 0x9E3779B97F4A7C15) & mask
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out


# --------------------------------------------------------------------------
# Named workloads.  Sizes and parameters follow the paper's runs (kT of order
# 1e-5..1e-4, gradients of order 1e-3, L of a few tens of nodes for physics)
# and the larger lattices used to measure throughput.
# --------------------------------------------------------------------------

def parity_small() -> Replica:
    """64 x 32, ideal mixture, all tau = 1, grad_c0 = 1e-3, kT = 1e-5, seed 1."""
    return Replica(Lx=64, Lz=32, grad_c0=1e-3, kT=1e-5, G=0.0, seed=1)


def single_512x256(grad_c0: float = 1e-3) -> Replica:
    """512 x 256 single lattice, G = 0.5, kT = 1e-5."""
    return Replica(Lx=512, Lz=256, grad_c0=grad_c0, kT=1e-5, G=0.5, seed=1)


def batched_ensemble(n: int = 96) -> List[Replica]:
    """96 replicas: L_i = 32 * 2^(i mod 4), Lx_i = 2 L_i; G_i = 0.5 when
    floor(i/4) is odd else 0; grad_c0_i = 1e-3 * u_i with u_i from SplitMix64
    seeded with 2018; Philox seed_i = 1 + i; tau = 1; kT = 1e-5."""
    draws = splitmix64(2018, n)
    reps = []
    for i in range(n):
        L = 32 * (2 ** (i % 4))
        u = (draws[i] >> 11) * (2.0 ** -53)
        reps.append(Replica(Lx=2 * L, Lz=L, grad_c0=1e-3 * u, kT=1e-5,
                            G=0.5 if (i // 4) % 2 == 1 else 0.0, seed=1 + i))
    return reps


def large_4096x1024() -> Replica:
    """4096 x 1024 single lattice, G = 0.5, grad_c0 = 5e-4, kT = 1e-5."""
    return Replica(Lx=4096, Lz=1024, grad_c0=5e-4, kT=1e-5, G=0.5, seed=1)


def adjoint_256x128() -> Replica:
    """256 x 128, G = 0.5, grad_c0 = 1e-3, kT = 1e-5, tau_s = 0.7, tau_d = 0.8."""
    return Replica(Lx=256, Lz=128, grad_c0=1e-3, kT=1e-5, G=0.5,
                   tau_s=0.7, tau_d=0.8, seed=1)
