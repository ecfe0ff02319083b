"""Seeded synthetic inputs for the two-phase DUGKS step: meshes, initial
fields and physical -> solver parameter helpers.

This module computes none of the scheme's arithmetic; it only builds the
arrays and the parameter dictionaries that both the HIP path and the test
oracle receive, so that the two see bit-identical inputs.

Test problems follow Sec. 3 of Zhang, Yang & Guo (arXiv:1802.02868):
stationary drop (Sec. 3.1, eq. droplet), layered Poiseuille flow on a
tanh-stretched mesh (Sec. 3.2, stretched-mesh formula), rising bubble
(Sec. 3.3, eq. dimensionless) and Rayleigh-Taylor instability (Sec. 3.4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RT_DEFAULT = 1.0 / 3.0  # Sec. 3: RT fixed at 1/3


def uniform_faces(n: int, x0: float = 0.0, dx: float = 1.0) -> np.ndarray:
    """n+1 equally spaced face coordinates starting at x0."""
    return x0 + dx * np.arange(n + 1, dtype=np.float64)


def stretched_faces(n: int, eps: float, half_width: float = 1.0) -> np.ndarray:
    """Face coordinates of the layered-Poiseuille mesh (Sec. 3.2): two tanh
    stretched halves, clustered at the walls y = +-H and at y = 0.

    Reading of the garbled index range: faces k = -n/2..n/2, with
    xi_k = +-1/2 + tanh(eps (k/(n/2) -+ 1/2)) / (2 tanh(eps/2)), y_k = H xi_k;
    cell centres are face midpoints."""
    if n % 2:
        raise ValueError("stretched mesh needs an even cell count")
    m = n // 2
    k = np.arange(-m, m + 1, dtype=np.float64)
    s = k / m
    t2 = 2.0 * math.tanh(eps / 2.0)
    xi = np.where(k >= 0, 0.5 + np.tanh(eps * (s - 0.5)) / t2,
                  -0.5 + np.tanh(eps * (s + 0.5)) / t2)
    xi[m] = 0.0
    xi[0], xi[-1] = -1.0, 1.0
    return half_width * xi


def centres(faces: np.ndarray) -> np.ndarray:
    return 0.5 * (faces[:-1] + faces[1:])


def beta_kappa(sigma: float, width: float, phi_a: float = 1.0, phi_b: float = 0.0):
    """Invert eqs. thickness and sigma: W = sqrt(8 kappa/beta)/(phi_A-phi_B),
    sigma = |phi_A-phi_B|^3 sqrt(2 kappa beta)/6."""
    d = abs(phi_a - phi_b)
    beta = 12.0 * sigma / (width * d ** 4)
    kappa = 1.5 * sigma * width / d ** 2
    return beta, kappa


def tanh_profile(dist, width, phi_a=1.0, phi_b=0.0):
    """Flat-interface equilibrium profile (eq. equilibriuminterface, first
    term read as (phi_A+phi_B)/2 as in eq. droplet); dist > 0 inside A."""
    return 0.5 * (phi_a + phi_b) + 0.5 * (phi_a - phi_b) * np.tanh(2.0 * np.asarray(dist) / width)


def bubble_numbers(g, rho_heavy, rho_light, diameter, sigma, mu_heavy):
    """Eotvos, Morton and Reynolds numbers of eq. dimensionless (fluid B is
    the surrounding heavy fluid)."""
    dr = rho_heavy - rho_light
    eo = g * dr * diameter ** 2 / sigma
    mo = g * dr * mu_heavy ** 4 / (rho_heavy ** 2 * sigma ** 3)
    re = math.sqrt(g * rho_heavy * dr * diameter ** 3) / mu_heavy
    return eo, mo, re


def bubble_scales(eo, mo, diameter, rho_l=1.0, rho_g=1e-3, u_ref=0.04):
    """Given Eo and Mo, fix sqrt(g D) = u_ref and solve eq. dimensionless for
    g, sigma and the liquid viscosity."""
    g = u_ref ** 2 / diameter
    dr = rho_l - rho_g
    sigma = g * dr * diameter ** 2 / eo
    mu_l = (mo * rho_l ** 2 * sigma ** 3 / (g * dr)) ** 0.25
    return g, sigma, mu_l / rho_l


@dataclass
class Case:
    """One synthetic problem: solver parameters plus initial fields."""
    name: str
    params: dict
    x_faces: np.ndarray
    y_faces: np.ndarray
    phi0: np.ndarray
    ux0: np.ndarray
    uy0: np.ndarray
    p0: np.ndarray
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def nx(self):
        return self.params["nx"]

    @property
    def ny(self):
        return self.params["ny"]


def base_params(**kw) -> dict:
    p = dict(nx=0, ny=0, bc_x=0, bc_y=0, recon=0, phi_clamp=0,
             cfl=0.0, c_max=0.0, dt=0.0, rt=RT_DEFAULT,
             tau_g=0.5, mobility=0.1, tau_f=0.0,
             beta=0.0, kappa=0.0, phi_a=1.0, phi_b=0.0, rho_a=1.0, rho_b=1.0,
             nu_a=0.1, nu_b=0.1, gx=0.0, gy=0.0, rho_ref=0.0)
    p.update(kw)
    return p


def drop_case(n=64, radius=16.0, width=4.0, sigma=1e-3, rho_a=1.0, rho_b=0.1, nu=0.1,
              mobility=0.1, cfl=0.5, c_max=1.0, noise=1e-6, seed=1234, steps=1000,
              tau_f=0.0, recon=0, centre=None) -> Case:
    """Stationary drop, periodic square, drop = fluid A (phi_A = 1)."""
    xf = uniform_faces(n)
    yf = uniform_faces(n)
    xc, yc = centres(xf), centres(yf)
    c0 = (n / 2.0, n / 2.0) if centre is None else centre
    X, Y = np.meshgrid(xc, yc)
    r = np.sqrt((X - c0[0]) ** 2 + (Y - c0[1]) ** 2)
    phi = tanh_profile(radius - r, width)
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        phi = phi + rng.uniform(-noise, noise, size=phi.shape)
    beta, kappa = beta_kappa(sigma, width)
    p = base_params(nx=n, ny=n, cfl=cfl, c_max=c_max, beta=beta, kappa=kappa,
                    rho_a=rho_a, rho_b=rho_b, nu_a=nu, nu_b=nu, mobility=mobility,
                    tau_f=tau_f, recon=recon)
    z = np.zeros_like(phi)
    return Case("drop%d" % n, p, xf, yf, np.ascontiguousarray(phi), z.copy(), z.copy(),
                z.copy(), steps, dict(radius=radius, sigma=sigma, width=width))


def tensor_drop_case(nx=32, ny=24, eps_x=1.5, eps_y=1.0, bc_x=1, bc_y=0, radius=None,
                     width=4.0, sigma=1e-3, rho_a=1.0, rho_b=0.1, nu=0.1, mobility=0.1,
                     cfl=0.4, gx=0.0, gy=0.0, steps=200) -> Case:
    """A drop on a general tensor mesh: both axes tanh-stretched like the
    layered-channel mesh (clustered at the ends and the middle), with walls
    or periodic ends per axis (default: walls in x, periodic in y).  Unit
    cells on average (half widths nx/2 and ny/2); the drop sits off-centre
    so that it meets fine and coarse cells."""
    xf = stretched_faces(nx, eps_x, nx / 2.0)
    yf = stretched_faces(ny, eps_y, ny / 2.0)
    xc, yc = centres(xf), centres(yf)
    r0 = min(nx, ny) / 5.0 if radius is None else radius
    X, Y = np.meshgrid(xc, yc)
    r = np.sqrt((X - 0.15 * nx) ** 2 + (Y + 0.1 * ny) ** 2)
    phi = tanh_profile(r0 - r, width)
    beta, kappa = beta_kappa(sigma, width)
    p = base_params(nx=nx, ny=ny, bc_x=bc_x, bc_y=bc_y, cfl=cfl, beta=beta, kappa=kappa,
                    rho_a=rho_a, rho_b=rho_b, nu_a=nu, nu_b=nu, mobility=mobility, gx=gx,
                    gy=gy, rho_ref=rho_b)
    z = np.zeros_like(phi)
    return Case("tensor%dx%d" % (nx, ny), p, xf, yf, np.ascontiguousarray(phi), z.copy(),
                z.copy(), z.copy(), steps, dict(radius=r0, sigma=sigma, width=width))


def poiseuille_case(nx=4, ny=128, eps=1.5, half=1.0, nu_a=0.01, nu_b=1.0, gx=1e-6,
                    width_cells=4.0, sigma=1e-4, mobility=1e-2, cfl=0.5, steps=1000,
                    stretched=True, recon=0) -> Case:
    """Layered Poiseuille flow between walls y = -H and y = H, fluid A below
    y = 0 and B above, driven by a body force along x."""
    yf = stretched_faces(ny, eps, half) if stretched else uniform_faces(ny, -half, 2 * half / ny)
    dy_min = float(np.min(np.diff(yf)))
    xf = uniform_faces(nx, 0.0, 2.0 * half / 128.0 if stretched else 2.0 * half / ny)
    width = width_cells * dy_min
    yc = centres(yf)
    phi1 = tanh_profile(-yc, width)
    phi = np.ascontiguousarray(np.tile(phi1[:, None], (1, nx)))
    beta, kappa = beta_kappa(sigma, width)
    p = base_params(nx=nx, ny=ny, bc_x=0, bc_y=1, cfl=cfl, beta=beta, kappa=kappa,
                    rho_a=1.0, rho_b=1.0, nu_a=nu_a, nu_b=nu_b, mobility=mobility,
                    gx=gx, rho_ref=0.0, recon=recon)
    z = np.zeros_like(phi)
    return Case("poiseuille%dx%d" % (nx, ny), p, xf, yf, phi, z.copy(), z.copy(), z.copy(),
                steps, dict(half=half, gx=gx, width=width))


def poiseuille_profile(y, half, gx, mu_a, mu_b):
    """Analytic layered Poiseuille profile (Sec. 3.2) with fluid A below y = 0
    (the paper's formula with y -> -y), body force gx playing G."""
    y = np.asarray(y, dtype=np.float64)
    s = -y / half
    r = (mu_a - mu_b) / (mu_a + mu_b)
    ua = gx * half ** 2 / (2 * mu_a) * (-s ** 2 - s * r + 2 * mu_a / (mu_a + mu_b))
    ub = gx * half ** 2 / (2 * mu_b) * (-s ** 2 - s * r + 2 * mu_b / (mu_a + mu_b))
    return np.where(s >= 0, ua, ub)


def rt_case(nx=256, ny=None, atwood=0.5, re=3000.0, pe=1000.0, sigma=5e-5, width=4.0,
            amp_frac=0.1, cfl=0.283, steps=20000, recon=0) -> Case:
    """Rayleigh-Taylor instability: heavy A (phi_A = 1) over light B, periodic
    in x, walls in y, domain nx x 4nx with the interface at mid height.
    U = sqrt(g nx) = 0.04; one dynamic viscosity mu = rho_A U nx / Re for
    both fluids (Sec. 3.4 defines Re with a single mu); mobility U nx / Pe
    (the section takes Re, Pe, sigma and W from a lattice Boltzmann study
    that it cites; the Peclet number is read as U L / lambda)."""
    ny = 4 * nx if ny is None else ny
    xf, yf = uniform_faces(nx), uniform_faces(ny)
    xc, yc = centres(xf), centres(yf)
    rho_b = 1.0
    rho_a = rho_b * (1 + atwood) / (1 - atwood)
    u_ref = 0.04
    g = u_ref ** 2 / nx
    mu = rho_a * u_ref * nx / re
    beta, kappa = beta_kappa(sigma, width)
    lam = u_ref * nx / pe
    X, Y = np.meshgrid(xc, yc)
    yi = ny / 2.0 + amp_frac * nx * np.cos(2 * np.pi * X / nx)
    phi = np.ascontiguousarray(tanh_profile(Y - yi, width))
    p = base_params(nx=nx, ny=ny, bc_x=0, bc_y=1, cfl=cfl, beta=beta, kappa=kappa,
                    rho_a=rho_a, rho_b=rho_b, nu_a=mu / rho_a, nu_b=mu / rho_b, mobility=lam,
                    gx=0.0, gy=-g, rho_ref=rho_b, recon=recon)
    z = np.zeros_like(phi)
    return Case("rt%dx%d" % (nx, ny), p, xf, yf, phi, z.copy(), z.copy(), z.copy(), steps,
                dict(g=g, mu=mu, lam=lam, width=width))


def bubble_case(nx, ny, eo, mo, rho_l=1.0, rho_g=0.1, visc_ratio=100.0, width=4.0,
                cfl=0.354, steps=5000, recon=0) -> Case:
    """Rising bubble in a closed box (four walls): bubble = fluid A (phi_A = 1,
    light), liquid = B.  Radius nx/8 centred at (nx/2, ny/4)."""
    xf, yf = uniform_faces(nx), uniform_faces(ny)
    xc, yc = centres(xf), centres(yf)
    d = nx / 4.0
    g, sigma, nu_l = bubble_scales(eo, mo, d, rho_l, rho_g)
    beta, kappa = beta_kappa(sigma, width)
    X, Y = np.meshgrid(xc, yc)
    r = np.sqrt((X - nx / 2.0) ** 2 + (Y - ny / 4.0) ** 2)
    phi = np.ascontiguousarray(tanh_profile(d / 2.0 - r, width))
    tau_g = 0.5
    lam = RT_DEFAULT * tau_g * 2.0  # eta = 2.0 as in Sec. 3.3
    p = base_params(nx=nx, ny=ny, bc_x=1, bc_y=1, cfl=cfl, beta=beta, kappa=kappa,
                    rho_a=rho_g, rho_b=rho_l, nu_a=nu_l / visc_ratio, nu_b=nu_l,
                    mobility=lam, tau_g=tau_g, gx=0.0, gy=-g, rho_ref=rho_l, phi_clamp=1,
                    recon=recon)
    z = np.zeros_like(phi)
    return Case("bubble%dx%d" % (nx, ny), p, xf, yf, phi, z.copy(), z.copy(), z.copy(),
                steps, dict(g=g, sigma=sigma, nu_l=nu_l, eo=eo, mo=mo))


def rt_mode_amplitudes(nx, nmodes=64, seed=2024, sigma_frac=1e-3):
    """Seeded amplitudes a_1..a_nmodes ~ N(0, (sigma_frac nx)^2) of the
    interface modes of the differentiable Rayleigh-Taylor rollout."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return sigma_frac * nx * rng.standard_normal(nmodes)


def rt_interface_phi0(amps, case):
    """Order parameter of a Rayleigh-Taylor interface at
    y_I(x) = ny/2 + sum_k a_k cos(2 pi k x / nx), k = 1..len(amps), with the
    tanh profile of the case's width (heavy fluid A above).  Accepts a numpy
    array or a torch tensor of amplitudes and returns the same kind (torch:
    differentiable, on the amplitudes' device)."""
    nx, ny = case.nx, case.ny
    width = case.meta.get("width", 4.0)
    xc, yc = centres(case.x_faces), centres(case.y_faces)
    k = np.arange(1, len(amps) + 1, dtype=np.float64)
    basis = np.cos(2.0 * np.pi * np.outer(k, xc) / nx)  # [modes, nx]
    if isinstance(amps, np.ndarray):
        yi = ny / 2.0 + amps @ basis
        return np.ascontiguousarray(tanh_profile(yc[:, None] - yi[None, :], width))
    import torch
    B = torch.as_tensor(basis, dtype=torch.float64, device=amps.device)
    Y = torch.as_tensor(yc, dtype=torch.float64, device=amps.device)
    yi = ny / 2.0 + amps @ B
    return (0.5 + 0.5 * torch.tanh(2.0 * (Y[:, None] - yi[None, :]) / width)).contiguous()


BUBBLE_SIZES = ((128, 256), (160, 320), (192, 384), (256, 512))


def bubble_batch(n=48, seed=4242, steps=5000):
    """48 rising bubbles with seeded sizes, Eo ~ U[10, 100], log10 Mo ~ U[-5, -1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        nx, ny = BUBBLE_SIZES[int(rng.integers(0, len(BUBBLE_SIZES)))]
        eo = float(rng.uniform(10.0, 100.0))
        mo = float(10.0 ** rng.uniform(-5.0, -1.0))
        c = bubble_case(nx, ny, eo, mo, steps=steps)
        c.name = "bubble%02d_%dx%d" % (k, nx, ny)
        out.append(c)
    return out


def drop_mass_median(phi, phi_a=1.0, phi_b=0.0):
    """Droplet mass by the median level of the order parameter (Sec. 3.1):
    number of cells with phi strictly above (phi_A + phi_B)/2."""
    return int(np.count_nonzero(np.asarray(phi) > 0.5 * (phi_a + phi_b)))


def table1_initial_phi(radius, n=100, width=4.0):
    """Initial drop of Table 1: 100 x 100 cells with centres at integer
    coordinates 0..99 and the drop centre at (50, 50)."""
    c = np.arange(n, dtype=np.float64)
    X, Y = np.meshgrid(c, c)
    r = np.sqrt((X - 50.0) ** 2 + (Y - 50.0) ** 2)
    return tanh_profile(radius - r, width)


def paper_drop_case(radius=25.0, cfl=0.4, mobility=0.1, steps=20000) -> Case:
    """The stationary drop as Sec. 3.1 sets it up: 100 x 100 periodic cells,
    rho_A = 1, rho_B = 0.2, tau_f = tau_g = 0.5, W = 4, sigma = 1e-3, CFL 0.4
    (C_max = sqrt(6 RT)); radius 10-40, mobility and CFL varied there."""
    c = drop_case(n=100, radius=radius, rho_a=1.0, rho_b=0.2, tau_f=0.5, mobility=mobility,
                  cfl=cfl, c_max=0.0, noise=0.0, steps=steps)
    c.name = "paper_drop100_r%g" % radius
    return c


def paper_channel_case(ratio=30.0, eps=None, mu_a=0.1, u_c=5e-5, steps=200000) -> Case:
    """The layered channel of Sec. 3.2: 10 x 200 cells between walls at
    y = -H, H (H = 100), fluid A above y = 0, mu_A / mu_B = ratio (3, 30, 100,
    1000 there), rho_A = rho_B = 1, W = 4, CFL 0.5, centre velocity
    u_c = G H^2 / (mu_A + mu_B) = 5e-5.  eps: the stretched mesh of the same
    section (2.5 there), else uniform.  The paper gives only the ratio, so
    mu_A = 0.1 is a reading."""
    half, ny, nx = 100.0, 200, 10
    yf = uniform_faces(ny, -half, 1.0) if eps is None else stretched_faces(ny, eps, half)
    xf = uniform_faces(nx)
    mu_b = mu_a / ratio
    g = u_c * (mu_a + mu_b) / half ** 2
    width = 4.0 * float(np.min(np.diff(yf)))
    beta, kappa = beta_kappa(1e-4, width)
    yc = centres(yf)
    phi = np.ascontiguousarray(np.tile(tanh_profile(yc, width)[:, None], (1, nx)))
    p = base_params(nx=nx, ny=ny, bc_x=0, bc_y=1, cfl=0.5, beta=beta, kappa=kappa,
                    rho_a=1.0, rho_b=1.0, nu_a=mu_a, nu_b=mu_b, mobility=1e-2, gx=g,
                    rho_ref=0.0)
    z = np.zeros_like(phi)
    name = "paper_channel10x200_ratio%g%s" % (ratio, "" if eps is None else "_eps%g" % eps)
    return Case(name, p, xf, yf, phi, z.copy(), z.copy(), z.copy(), steps,
                dict(half=half, gx=g, mu_a=mu_a, mu_b=mu_b, width=width))


def paper_bubble_case(ratio=2, steps=20000) -> Case:
    """The rising bubble as Sec. 3.3 sets it up: an L0 x 3 L0 periodic box,
    L0 = 160, a light bubble (fluid A) of diameter D = 2 L0 / 5 at
    (L0/2, L0/2), buoyancy -(rho - rho_B) G_y with G_y = 1e-5, sigma = 1e-3,
    eta = 2.0, tau_f = tau_g = 0.5 (viscosity ratio 1), W = 4, CFL 0.354.
    rho_B / rho_A = 2 or 5; the absolute densities are the reading that
    reproduces the Eo, Mo, Re printed for the two runs."""
    l0 = 160
    rho_b, rho_a = {2: (1.0, 0.5), 5: (1.2, 0.24)}[int(ratio)]
    xf, yf = uniform_faces(l0), uniform_faces(3 * l0)
    xc, yc = centres(xf), centres(yf)
    X, Y = np.meshgrid(xc, yc)
    r = np.sqrt((X - l0 / 2.0) ** 2 + (Y - l0 / 2.0) ** 2)
    phi = np.ascontiguousarray(tanh_profile(l0 / 5.0 - r, 4.0))
    beta, kappa = beta_kappa(1e-3, 4.0)
    tau_g = 0.5
    p = base_params(nx=l0, ny=3 * l0, bc_x=0, bc_y=0, cfl=0.354, beta=beta, kappa=kappa,
                    rho_a=rho_a, rho_b=rho_b, tau_f=0.5, tau_g=tau_g,
                    mobility=RT_DEFAULT * tau_g * 2.0, gx=0.0, gy=-1e-5, rho_ref=rho_b)
    z = np.zeros_like(phi)
    return Case("paper_bubble160x480_ratio%d" % ratio, p, xf, yf, phi, z.copy(), z.copy(),
                z.copy(), steps, dict(diameter=2 * l0 / 5.0, g=1e-5))


def paper_rt_case(atwood=0.1, re=3000.0, steps=20000) -> Case:
    """Rayleigh-Taylor as Sec. 3.4 sets it up: d = L = 256 on [0, d] x
    [-2d, 2d], walls top and bottom, periodic sides, interface
    2d + 0.05 d cos(2 pi x / L), Re = 3000 (150 in the same figure's first
    row), sqrt(g L) = 0.04, W = 4, sigma = 5e-5; At = 0.1 with CFL 0.35, or
    At = 0.5 with CFL 0.283."""
    cfl = 0.35 if atwood < 0.3 else 0.283
    c = rt_case(256, atwood=atwood, re=re, amp_frac=0.05, cfl=cfl, steps=steps)
    c.name = "paper_rt256x1024_at%g%s" % (atwood, "" if re == 3000.0 else "_re%g" % re)
    return c


PAPER_CASES = {
    "paper_drop100_r25": lambda: paper_drop_case(25.0),
    "paper_drop100_r10": lambda: paper_drop_case(10.0),
    "paper_channel10x200_ratio3": lambda: paper_channel_case(3.0),
    "paper_channel10x200_ratio1000": lambda: paper_channel_case(1000.0),
    "paper_channel10x200_ratio30_eps2.5": lambda: paper_channel_case(30.0, eps=2.5),
    "paper_bubble160x480_ratio2": lambda: paper_bubble_case(2),
    "paper_bubble160x480_ratio5": lambda: paper_bubble_case(5),
    "paper_rt256x1024_at0.1": lambda: paper_rt_case(0.1),
    "paper_rt256x1024_at0.1_re150": lambda: paper_rt_case(0.1, re=150.0),
}


def config(name: str) -> Case:
    """Named workloads: the drop (Sec. 3.1), the layered channel (Sec. 3.2)
    and Rayleigh-Taylor (Sec. 3.4) at 256 x 1024 and 512 x 2048."""
    if name == "drop64":
        return drop_case()
    if name == "poiseuille4x128":
        return poiseuille_case(steps=250000)
    if name == "rt256x1024":
        return rt_case(256)
    if name == "rt512x2048":
        return rt_case(512, steps=2000)
    raise KeyError(name)
