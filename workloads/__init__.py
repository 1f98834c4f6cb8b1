"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module only draws random physical parameters (numpy PCG64 via
``default_rng(seed)``) and states the fixed constants of each workload.  It
holds none of the method's arithmetic: no eigenvalues, no coupling tensors, no
scheme coefficients and no geometry solves.  Whatever a workload leaves to be
derived (for example a plate area chosen so that the highest simulated mode
sits at a given frequency) is named here as a target and derived separately by
each consumer.

The workloads follow the paper's own experiments (Sec. 4.2 benchmarks: von
Karman and tension-modulated models at 10/50/100 modes, 1 s at 44.1 kHz;
Sec. 4.3 inverse modelling) at the sizes of the five benchmark configurations.
"""
from __future__ import annotations

import numpy as np

FS = 44100.0

# steel, the material of the single-plate workload
STEEL = dict(E=2e11, nu=0.3, rho=7860.0)


def string_kc(seed: int = 1, n_modes: int = 30, n_steps: int = 22050) -> dict:
    """Tension-modulated (Kirchhoff-Carrier) string, 0.65 m, 30 sine modes.

    Raised-cosine pluck of 1 mm amplitude and total width 0.1 L, centred at a
    seeded position in [0.1 L, 0.4 L]; output at a seeded point in
    [0.1 L, 0.9 L].  Damping law sigma_k = 1 + 0.002 omega_k (rate, 1/s).
    """
    rng = np.random.default_rng(seed)
    L = 0.65
    x_pluck = rng.uniform(0.1 * L, 0.4 * L)
    x_out = rng.uniform(0.1 * L, 0.9 * L)
    return dict(
        family="string", model="kc", L=L, T0=60.0, rhoA=6e-4, EA=3e5, EI=0.0,
        n_modes=n_modes, fs=FS, n_steps=n_steps,
        damping=("affine_omega", 1.0, 0.002),
        pluck=dict(x0=x_pluck, amplitude=1e-3, width=0.1 * L),
        x_out=x_out, proj_cells=4096,
    )


def plate_vk(seed: int = 2, n_t: int = 40, n_in: int | None = None,
             n_steps: int = 44100, family: str = "clamped",
             grid=(200, 150), proj_grid=None) -> dict:
    """Single von Karman plate, 0.4 x 0.3 m steel, 1 mm, simply supported.

    Strike: raised-cosine initial displacement of seeded height in
    [0.5 h, 3 h] and radius 0.1 min(Lx, Ly); strike centre and output point
    drawn independently in [0.1, 0.9] x (Lx, Ly).  No pre-tension.
    ``grid``: midpoint grid of the coupling integrals (None = exact, sine
    family only); ``proj_grid``: grid of the strike projection (default: the
    coupling grid, else 200 x 150).
    """
    rng = np.random.default_rng(seed)
    h = 1e-3
    Lx, Ly = 0.4, 0.3
    amp = rng.uniform(0.5, 3.0) * h
    cx, cy = rng.uniform(0.1, 0.9, size=2)
    ox, oy = rng.uniform(0.1, 0.9, size=2)
    return dict(
        family="plate", model="vk", inplane=family, Lx=Lx, Ly=Ly, h=h,
        T0=0.0, **STEEL, n_t=n_t, n_in=n_t if n_in is None else n_in,
        fs=FS, n_steps=n_steps, grid=None if grid is None else tuple(grid),
        damping=("affine_omega", 1.0, 0.002),
        strike=dict(xc=cx * Lx, yc=cy * Ly, amplitude=amp,
                    radius=0.1 * min(Lx, Ly)),
        out=(ox * Lx, oy * Ly),
        proj_grid=tuple(proj_grid or grid or (200, 150)),
    )


def plate_batch(seed: int = 3, batch: int = 256, n_lo: int = 50,
                n_hi: int = 400, n_steps: int = 44100,
                top_mode_hz: float = 5000.0) -> list[dict]:
    """Batch of uneven von Karman plates for one persistent launch.

    Transverse mode count N_b ~ U{n_lo..n_hi}, in-plane count equal to it;
    aspect Ly/Lx ~ U[0.5, 1]; thickness ~ U[0.5, 2] mm; Young's modulus and
    pre-tension log-uniform over one decade (centred on steel's 2e11 Pa;
    10..100 N/m).  The plate area is left to the consumer: it is the one that
    puts transverse mode N_b at ``top_mode_hz``.  Coupling tensors use the
    sine in-plane family with exact integrals.  Strike height ~ U[0.5, 3] h,
    radius 0.1 min(Lx, Ly); centre and output point ~ U[0.1, 0.9]^2 of the
    plate.
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(batch):
        n = int(rng.integers(n_lo, n_hi + 1))
        aspect = float(rng.uniform(0.5, 1.0))
        h = float(rng.uniform(0.5e-3, 2e-3))
        E = float(2e11 * 10.0 ** rng.uniform(-0.5, 0.5))
        T0 = float(10.0 ** rng.uniform(1.0, 2.0))
        amp = float(rng.uniform(0.5, 3.0)) * h
        cx, cy, ox, oy = (float(v) for v in rng.uniform(0.1, 0.9, size=4))
        out.append(dict(
            family="plate", model="vk", inplane="sine", grid=None,
            aspect=aspect, top_mode_hz=top_mode_hz, h=h, E=E, nu=0.3,
            rho=7860.0, T0=T0, n_t=n, n_in=n, fs=FS, n_steps=n_steps,
            damping=("affine_omega", 1.0, 0.002),
            strike_rel=dict(xc=cx, yc=cy, amplitude=amp, radius_rel=0.1),
            out_rel=(ox, oy), proj_grid=(256, 256), index=b,
        ))
    return out


def plate_sweep(n_t: int, seed: int = 2, n_steps: int = 44100) -> dict:
    """The paper's benchmark shapes: the single-plate geometry at 10/50/100
    modes (Sec. 4.2, Fig. 2), sine in-plane family, 1 s at 44.1 kHz."""
    return plate_vk(seed=seed, n_t=n_t, n_steps=n_steps, family="sine")


def plate_fit(seed: int = 4, n_t: int = 200, n_in: int | None = None, n_steps: int = 44100,
              perturb: float = 0.1) -> dict:
    """Parameter fitting of one von Karman plate (steel, 1 mm, area 0.12 m^2,
    base aspect 0.75, i.e. 0.4 x 0.3 m) by gradients through the time loop.

    theta = (T0/rho_s, D/rho_s, aspect Ly/Lx, d1/(2 rho_s), d3/(2 rho_s)).
    The base point has T0 = 50 N/m, steel's bending stiffness, d1^ = 1 /s and
    d3^ such that the damping of a 5 kHz mode is about 50 /s; the target
    parameters are the base ones times exp(U[-perturb, perturb]) each
    (seeded).  Strike 1 h at a fixed relative position; pickup fixed.
    """
    rng = np.random.default_rng(seed)
    h, rho, E, nu = 1e-3, 7860.0, 2e11, 0.3
    rho_s = rho * h
    D = E * h ** 3 / (12 * (1 - nu ** 2))
    base = np.array([50.0 / rho_s, D / rho_s, 0.75, 1.0, 0.0])
    # d3^ lambda at 5 kHz ~ 49 /s: lambda from omega^2 = D^ lambda^2 + T0^ lambda
    w = 2 * np.pi * 5000.0
    lam5 = (-base[0] + np.sqrt(base[0] ** 2 + 4 * base[1] * w * w)) / (2 * base[1])
    base[4] = 49.0 / lam5
    target = base * np.exp(rng.uniform(-perturb, perturb, size=5))
    return dict(n_t=n_t, n_in=n_t if n_in is None else n_in, area=0.12, h=h, nu=nu, rho=rho,
                base_aspect=0.75, strike=(0.37, 0.61, 1.0 * h, 0.1), out=(0.71, 0.29),
                proj_grid=(200, 150), fs=FS, n_steps=n_steps, theta0=base, theta_target=target)


def string_fit(seed: int = 7, n_modes: int = 20, n_steps: int = 11025, perturb: float = 0.1) -> dict:
    """Parameter fitting of one Kirchhoff-Carrier string by gradients through
    the time loop.

    theta = (T0/rhoA, EI/rhoA, L, d1^, d3^) with gamma_k = d1^ + d3^ lambda_k.
    The base point is the 0.65 m, 60 N, 6e-4 kg/m string (T0^ = 1e5) with a
    light bending stiffness (EI^ = 0.2, inharmonicity about 1e-5), d1^ = 1 /s
    and d3^ such that the 20th mode (about 4.9 kHz) decays at about 57 /s;
    EA/rhoA = 5e8 fixed.  Pluck at 0.27 L, 1 mm, width 0.1 L; pickup at
    0.71 L.  The target is the base times exp(U[-perturb, perturb]) each
    (seeded)."""
    rng = np.random.default_rng(seed)
    base = np.array([1e5, 0.2, 0.65, 1.0, 6e-3])
    target = base * np.exp(rng.uniform(-perturb, perturb, size=5))
    return dict(n_modes=n_modes, EAhat=5e8, pluck=(0.27, 1e-3, 0.1), out=0.71, proj_cells=4096,
                fs=FS, n_steps=n_steps, theta0=base, theta_target=target)


def plate_group(seed: int = 6, batch: int = 48, n_t: int = 40, n_in: int | None = None,
                n_steps: int = 44100, forced: int = 0) -> dict:
    """A group of plates that share one coupling tensor up to per-row scales.

    Base: the sine-family plate of ``plate_vk`` (exact integrals).  Member b
    scales in-plane row n of the base's scaled tensor by row_scale[b][n]
    ~ U[0.5, 1.5] (as a change of stiffness or of in-plane eigenvalues would),
    its angular frequencies by U[0.97, 1.03] and decay rates by U[0.8, 1.25]
    (one factor per member), and its initial displacement by U[0.5, 1.5].
    The first ``forced`` members are also driven: b_ext ~ N(0, 1) per mode
    (scaled by 10, displacements well under the thickness) times a seeded
    noise burst of 2000 samples.
    """
    rng = np.random.default_rng(seed)
    base = plate_vk(seed=seed + 1000, n_t=n_t, n_in=n_in, family="sine", grid=None,
                    n_steps=n_steps)
    members = []
    for b in range(batch):
        m = dict(row_scale=rng.uniform(0.5, 1.5, size=base["n_in"]),
                 omega_factor=float(rng.uniform(0.97, 1.03)),
                 gamma_factor=float(rng.uniform(0.8, 1.25)),
                 amp_factor=float(rng.uniform(0.5, 1.5)))
        if b < forced:
            m["b_ext"] = 10.0 * rng.normal(size=n_t)
            m["e_ext"] = rng.normal(size=2000).astype(np.float32)
        members.append(m)
    return dict(base=base, members=members, n_steps=n_steps, fs=FS)


def plate_berger(seed: int = 2, n_t: int = 40, n_steps: int = 44100) -> dict:
    """Tension-modulated (Berger) plate: the single plate's geometry,
    material, damping and seeded strike/pickup (``plate_vk``), with the
    nonlinearity of the tension equation instead of von Karman coupling."""
    wl = plate_vk(seed=seed, n_t=n_t, n_in=0, n_steps=n_steps, family="sine", grid=None)
    wl["model"] = "berger"
    return wl


def linear_batch(seed: int = 9, batch: int = 64, n_modes: int = 60, n_steps: int = 44100,
                 forced: int = 8) -> dict:
    """Linear (stiff) strings for the closed-form path: fundamental
    f0 ~ U[80, 800] Hz, inharmonicity B ~ U[0, 1e-4] (f_k = k f0 sqrt(1 + B k^2)),
    modes kept below 12 kHz; decay rates gamma_k = s0 + s2 omega_k^2 with
    s0 ~ U[0.5, 3] /s and s2 ~ U[0.5, 5] 1e-8 s; released from rest with
    q^0_k = sin(k pi x_p) / k^2 for x_p ~ U[0.1, 0.4] (scaled to 1 mm);
    pickup c_k = sin(k pi x_o), x_o ~ U[0.5, 0.9]; the first `forced` strings
    are also driven by b_k = sin(k pi x_e) times a 1000-sample noise burst."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(batch):
        f0 = rng.uniform(80, 800)
        B = rng.uniform(0, 1e-4)
        k = np.arange(1, n_modes + 1)
        f = k * f0 * np.sqrt(1 + B * k * k)
        k = k[f < 12000.0]
        f = f[f < 12000.0]
        w = 2 * np.pi * f
        s0, s2 = rng.uniform(0.5, 3.0), rng.uniform(0.5, 5.0) * 1e-8
        xp, xo, xe = rng.uniform(0.1, 0.4), rng.uniform(0.5, 0.9), rng.uniform(0.1, 0.9)
        x0 = 1e-3 * np.sin(k * np.pi * xp) / k ** 2
        inst = dict(kind="linear", omega=w, gamma=s0 + s2 * w * w, x0=x0, xm1=x0.copy(),
                    c=np.sin(k * np.pi * xo))
        if b < forced:
            inst["b_ext"] = np.sin(k * np.pi * xe)
            inst["e_ext"] = (1e3 * rng.normal(size=1000)).astype(np.float32)
        out.append(inst)
    return dict(instances=out, n_steps=n_steps, fs=FS)
