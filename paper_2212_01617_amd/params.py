"""Lattice parameters from the non-dimensional groups of the droplet runs.

Sec. 3.1 defines Re = gamma a^2 / nu, Ca = a gamma mu_c / sigma,
Pe = gamma a xi / (M A), Ch = xi / a; Sec. 2.2 gives nu = cs^2 (tau_f - 1/2)
and M = Gamma (tau_g - 1/2).  For the symmetric binary free energy
A/4 (phi^2 - 1)^2 + kappa/2 |grad phi|^2 the interface width is
xi = sqrt(kappa/A) and the tension sigma = sqrt(8 kappa A / 9), so
A = 3 sigma / (2 sqrt(2) xi) and kappa = A xi^2.

Stability of the explicit Cahn-Hilliard update: with tau_g = 1 one step
changes phi by (Gamma/2) lap_h mu, and mu contains -kappa lap_h phi; the
odd-even mode (|lap_h| up to 16/3 on D2Q9 and D3Q19) is amplified by
|1 - Gamma kappa lap^2 / 2| and grows once Gamma kappa exceeds about 0.14.
derive_params keeps the mobility M that Pe asks for and, when
Gamma kappa would exceed `gk_max`, raises tau_g so that
Gamma = M / (tau_g - 1/2) = gk_max / kappa.
"""
from __future__ import annotations

import math
from dataclasses import asdict, dataclass

CS2 = 1.0 / 3.0


@dataclass
class DropletParams:
    A: float
    kappa: float
    M: float
    tau_f: float
    tau_g: float
    sigma: float
    xi: float
    rate: float       # shear rate gamma (or extension rate epsilon)
    wall_u: float     # shear: wall speed u_w = gamma H / 2
    nu: float

    def phys(self) -> dict:
        return dict(A=self.A, kappa=self.kappa, M=self.M, tau_f=self.tau_f, tau_g=self.tau_g)

    def as_dict(self) -> dict:
        return asdict(self)


def derive_params(*, Re: float, Ca: float, radius: float, xi: float, H: float = 0.0,
                  Pe: float = 0.43, tau_f: float = 1.0, M: float | None = None,
                  gk_max: float = 0.1) -> DropletParams:
    nu = CS2 * (tau_f - 0.5)
    rate = Re * nu / radius ** 2
    sigma = radius * rate * nu / Ca          # rho = 1: mu_c = nu
    A = 3.0 * sigma / (2.0 * math.sqrt(2.0) * xi)
    kappa = A * xi * xi
    if M is None:
        M = rate * radius * xi / (Pe * A)
    tau_g = 1.0
    if (M / (tau_g - 0.5)) * kappa > gk_max:
        tau_g = 0.5 + M * kappa / gk_max
    return DropletParams(A=A, kappa=kappa, M=M, tau_f=tau_f, tau_g=tau_g, sigma=sigma, xi=xi,
                         rate=rate, wall_u=rate * H / 2.0, nu=nu)
