"""Physical-parameter fitting through the GPU time loop.

Paper, Sec. 4.3: parameters are fitted by propagating gradients through the
time integrator (BPTT), in density-normalised form (D^ = D/rho_s,
T0^ = T0/rho_s), with the damping kept in the stable half plane, using Adam
with a one-cycle cosine learning-rate schedule and a spectral loss.

A plate here has five parameters theta = (T0^, D^, a, d1^, d3^):
    omega_k^2 = D^ lambda_k^2 + T0^ lambda_k,   gamma_k = d1^ + d3^ lambda_k,
    lambda_k  = pi^2 (m_k^2 a / S + q_k^2 / (a S))   (Lx = sqrt(S/a), Ly = sqrt(S a)),
with the area S, thickness, Poisson ratio, strike and pickup (relative
positions) fixed, and the mode index sets fixed at the base aspect so that
derivatives do not cross mode reorderings.  The von Karman prefactor follows
the bending stiffness: E/(2 rho) = 6 (1 - nu^2) D^ / h^2.  For the sine
in-plane family the unscaled coupling integrals at fixed area do not depend
on a (the Lx, Ly factors cancel), so the coupling tensor's aspect tangent is
a per-row rescaling through zeta_n^2 = lambda_n(a).

``ModalFn`` is a torch.autograd.Function whose forward runs modal_run and
whose backward runs modal_grad, followed by the FP64 chain rule to theta.

A tension-modulated (Kirchhoff-Carrier) string has five parameters too,
theta = (T0^, EI^, L, d1^, d3^) with T0^ = T0/(rho A), EI^ = EI/(rho A):
    omega_k^2 = EI^ lambda_k^2 + T0^ lambda_k,   gamma_k = d1^ + d3^ lambda_k,
    lambda_k  = (k pi / L)^2,   kappa = EA^/(2 L)   (Sec. 3: tau = EA/(2L)),
with EA^ = EA/(rho A), the pluck and the pickup (relative positions) fixed.
Its nonlinear force kappa lambda_k q_k sum_j lambda_j q_j^2 scales as L^-5
when L changes (kappa as 1/L, every lambda as 1/L^2), so the length enters the
force through the force-scale gradient.  ``StringFn`` is its autograd
function.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import modal, physics
from .losses import mrstft_loss

PARAM_NAMES = ("T0hat", "Dhat", "aspect", "d1hat", "d3hat")


@dataclass
class PlateSetup:
    """Fixed part of a fitted plate."""
    n_t: int = 200
    n_in: int = 200
    area: float = 0.12
    h: float = 1e-3
    nu: float = 0.3
    base_aspect: float = 0.75
    strike: tuple = (0.37, 0.61, 1e-3, 0.1)   # xc/Lx, yc/Ly, amplitude, radius/min(Lx,Ly)
    out: tuple = (0.71, 0.29)                   # xo/Lx, yo/Ly
    proj_grid: tuple = (200, 150)
    fs: float = 44100.0
    modes: tuple = field(default=None, repr=False)  # (m, q, a_in, b_in) at base aspect

    def __post_init__(self):
        if self.modes is None:
            Lx, Ly = math.sqrt(self.area / self.base_aspect), math.sqrt(self.area * self.base_aspect)
            m, q, _ = physics.plate_eigs(Lx, Ly, self.n_t)
            a, b, _ = physics.plate_eigs(Lx, Ly, self.n_in)
            self.modes = (m, q, a, b)


def _lam(m, q, aspect, area):
    return np.pi ** 2 * (m ** 2 * aspect / area + q ** 2 / (aspect * area))


def _dlam_da(m, q, aspect, area):
    return np.pi ** 2 * (m ** 2 / area - q ** 2 / (aspect ** 2 * area))


def _excitation(setup, aspect):
    m, q, _, _ = setup.modes
    Lx, Ly = math.sqrt(setup.area / aspect), math.sqrt(setup.area * aspect)
    xc, yc, amp, rr = setup.strike
    x0 = physics.plate_initial(m, q, Lx, Ly, setup.proj_grid, xc * Lx, yc * Ly, amp,
                               rr * min(Lx, Ly))
    c = physics.plate_pickup(m, q, Lx, Ly, setup.out[0] * Lx, setup.out[1] * Ly)
    return x0, c


def plate_instance(setup: PlateSetup, theta, threads=0):
    """Instance dict for theta = (T0^, D^, a, d1^, d3^), plus the pieces the
    chain rule needs."""
    T0h, Dh, a, d1, d3 = (float(v) for v in theta)
    m, q, ai, bi = setup.modes
    Lx, Ly = math.sqrt(setup.area / a), math.sqrt(setup.area * a)
    lam = _lam(m, q, a, setup.area)
    omega = np.sqrt(Dh * lam ** 2 + T0h * lam)
    gamma = d1 + d3 * lam
    zeta2 = _lam(ai, bi, a, setup.area)
    pref = math.sqrt(6.0 * (1.0 - setup.nu ** 2) * Dh / setup.h ** 2)
    Ht = modal.vk_coupling_sine(Lx, Ly, m, q, ai, bi, pref / zeta2, grid=None, threads=threads)
    x0, c = _excitation(setup, a)
    return dict(kind="vk", omega=omega, gamma=gamma, lam=lam, Ht=Ht, x0=x0, xm1=x0.copy(), c=c,
                zeta2=zeta2)


_BASE_TENSORS = {}
_EXCITATIONS = {}


def _excitation_cached(setup, aspect):
    """Strike projection and pickup per (setup, aspect), kept for batches
    drawn from a grid of aspect ratios (copies are returned)."""
    key = (id(setup), float(aspect))
    if key not in _EXCITATIONS:
        if len(_EXCITATIONS) > 4096:
            _EXCITATIONS.clear()
        _EXCITATIONS[key] = (setup, _excitation(setup, aspect))
    x0, c = _EXCITATIONS[key][1]
    return x0.copy(), c.copy()


def base_tensor(setup: PlateSetup):
    """Unscaled sine-family coupling tensor of the setup's mode sets (float32,
    one object per setup, cached): at fixed area it is the same for every
    aspect ratio."""
    key = (id(setup), setup.area)
    if key not in _BASE_TENSORS:
        m, q, ai, bi = setup.modes
        Lx, Ly = math.sqrt(setup.area / setup.base_aspect), math.sqrt(setup.area * setup.base_aspect)
        _BASE_TENSORS[key] = (setup, modal.vk_coupling_sine(Lx, Ly, m, q, ai, bi, np.ones(len(ai)),
                                                            grid=None))
    return _BASE_TENSORS[key][1]


def plate_instance_shared(setup: PlateSetup, theta):
    """The plate of ``plate_instance`` expressed as the setup's base tensor
    with per-row scales pref / zeta_n^2(a): batches of such instances share
    one tensor and run on the library's dense (MFMA) path."""
    T0h, Dh, a, d1, d3 = (float(v) for v in theta)
    m, q, ai, bi = setup.modes
    lam = _lam(m, q, a, setup.area)
    omega = np.sqrt(Dh * lam ** 2 + T0h * lam)
    gamma = d1 + d3 * lam
    zeta2 = _lam(ai, bi, a, setup.area)
    pref = math.sqrt(6.0 * (1.0 - setup.nu ** 2) * Dh / setup.h ** 2)
    x0, c = _excitation_cached(setup, a)
    return dict(kind="vk", omega=omega, gamma=gamma, lam=lam, Ht=base_tensor(setup),
                h_row_scale=pref / zeta2, x0=x0, xm1=x0.copy(), c=c, zeta2=zeta2)


def aspect_tangent(setup, inst, a):
    """dHt/da: row n of Ht scales as 1/zeta_n^2(a)."""
    _, _, ai, bi = setup.modes
    kappa = -_dlam_da(ai, bi, a, setup.area) / inst["zeta2"]
    return (inst["Ht"] * kappa[:, None, None].astype(np.float32)).astype(np.float32)


def chain_rule(setup, theta, inst, g, h_rel=1e-6):
    """dL/dtheta from the per-mode gradients of modal_grad (one instance)."""
    T0h, Dh, a, d1, d3 = (float(v) for v in theta)
    m, q, _, _ = setup.modes
    lam, om = inst["lam"], inst["omega"]
    gw, gg = g["omega"], g["gamma"]
    dlam = _dlam_da(m, q, a, setup.area)
    dT0 = np.sum(gw * lam / (2 * om))
    dD = np.sum(gw * lam ** 2 / (2 * om)) + g["scale"] / Dh
    dd1 = np.sum(gg)
    dd3 = np.sum(gg * lam)
    # aspect: frequencies, damping, coupling rows, excitation and pickup; the
    # coupling rows scale as 1/zeta_n^2(a), so with per-row gradients
    # dL/d log s_n the tensor term is sum_n (d log s_n/da) dL/d log s_n
    if g.get("row") is not None and len(g["row"]):
        _, _, ai, bi = setup.modes
        kappa = -_dlam_da(ai, bi, a, setup.area) / _lam(ai, bi, a, setup.area)
        tensor_term = float(np.sum(kappa * g["row"]))
    else:
        tensor_term = g["theta"]
    da = np.sum(gw * (2 * Dh * lam + T0h) * dlam / (2 * om)) + np.sum(gg * d3 * dlam) + tensor_term
    eps = h_rel * a
    xp, cp = _excitation(setup, a + eps)
    xm, cm = _excitation(setup, a - eps)
    da += np.sum((g["x0"] + g["xm1"]) * (xp - xm) / (2 * eps)) + np.sum(g["c"] * (cp - cm) / (2 * eps))
    return np.array([dT0, dD, da, dd1, dd3])


class ModalFn(torch.autograd.Function):
    """y = simulate(theta) for a batch of parameter vectors (one plate each).
    forward: modal_init + modal_run; backward: modal_grad + chain rule."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, setup: PlateSetup, n_steps: int, ckpt: int = 512):
        th = theta.detach().double().cpu().numpy().reshape(-1, 5)
        # base tensor + row scales: no per-plate tensor build; the library
        # stores each plate's scaled copy for the gradient kernels
        insts = [plate_instance_shared(setup, t) for t in th]
        sim = modal.Sim(insts, setup.fs, flags=modal.FLAG_GRAD)
        y = sim.run(n_steps).clone()
        ctx.save = (sim, insts, th, setup, n_steps, ckpt)
        return y

    @staticmethod
    def backward(ctx, gy):
        sim, insts, th, setup, n_steps, ckpt = ctx.save
        # the aspect derivative of the tensor is a per-row rescaling, taken
        # from the per-row gradients (no tangent tensor)
        g = sim.grad(n_steps, gy.contiguous().float(), ckpt_every=ckpt)
        # the per-plate chain rules (each projects the strike at two aspects)
        # run on host threads; numpy releases the interpreter lock in them
        def one(b):
            return chain_rule(setup, th[b], insts[b], {k: v[b] for k, v in g.items()})
        with ThreadPoolExecutor(max_workers=max(1, min(16, len(insts), os.cpu_count() or 1))) as ex:
            out = np.stack(list(ex.map(one, range(len(insts)))))
        sim.close()
        return torch.tensor(out, dtype=torch.float64).reshape(-1, 5), None, None, None


def one_cycle_cosine(step, total, peak, warm_frac=0.3, div=25.0, final_div=1e4):
    """One-cycle schedule: cosine rise from peak/div to peak over the first
    warm_frac of the steps, then cosine decay to peak/final_div."""
    w = max(1, int(warm_frac * total))
    if step < w:
        t = step / w
        lo = peak / div
        return lo + (peak - lo) * 0.5 * (1 - math.cos(math.pi * t))
    t = (step - w) / max(1, total - w)
    lo = peak / final_div
    return lo + (peak - lo) * 0.5 * (1 + math.cos(math.pi * t))


def to_unconstrained(theta, bounds=(0.3, 1.5)):
    """theta -> z: logs of the positive parameters, logit of the geometry
    parameter (a plate's aspect ratio, a string's length) in `bounds`
    (keeps gamma > 0 and the instance non-degenerate)."""
    lo, hi = bounds
    t = np.asarray(theta, float)
    z = np.log(t.copy())
    z[2] = math.log((t[2] - lo) / (hi - t[2]))
    return z


def from_unconstrained(z, bounds=(0.3, 1.5)):
    lo, hi = bounds
    z = torch.as_tensor(z)
    t = torch.exp(z)
    a = lo + (hi - lo) * torch.sigmoid(z[..., 2])
    return torch.cat([t[..., :2], a[..., None], t[..., 3:]], dim=-1)


# ------------------------------------------------------------------ strings
STRING_PARAM_NAMES = ("T0hat", "EIhat", "length", "d1hat", "d3hat")


@dataclass
class StringSetup:
    """Fixed part of a fitted Kirchhoff-Carrier string."""
    n_modes: int = 20
    EAhat: float = 5e8                  # EA / (rho A): the 3e5 N, 6e-4 kg/m string
    pluck: tuple = (0.27, 1e-3, 0.1)    # x / L, amplitude, total width / L
    out: float = 0.71                   # pickup x / L
    proj_cells: int = 4096
    fs: float = 44100.0
    bounds: tuple = (0.3, 1.2)          # length range of the unconstrained fit


_STRING_EXC = {}


def _string_excitation(setup, L):
    """Pluck projection and pickup weights at length L (cached per length)."""
    key = (id(setup), float(L))
    if key not in _STRING_EXC:
        if len(_STRING_EXC) > 4096:
            _STRING_EXC.clear()
        k = np.arange(1, setup.n_modes + 1, dtype=np.float64)
        xp, amp, w = setup.pluck
        x0 = physics.string_initial(k, L, dict(x0=xp * L, amplitude=amp, width=w * L), setup.proj_cells)
        c = math.sqrt(2.0 / L) * np.sin(k * np.pi * setup.out)
        _STRING_EXC[key] = (setup, (x0, c))
    x0, c = _STRING_EXC[key][1]
    return x0.copy(), c.copy()


def string_instance(setup: StringSetup, theta):
    """Instance dict (kind tension) for theta = (T0^, EI^, L, d1^, d3^)."""
    T0h, EIh, L, d1, d3 = (float(v) for v in theta)
    _, lam = physics.string_eigs(L, setup.n_modes)
    omega = np.sqrt(EIh * lam ** 2 + T0h * lam)
    gamma = d1 + d3 * lam
    x0, c = _string_excitation(setup, L)
    return dict(kind="tension", omega=omega, gamma=gamma, lam=lam, kappa=setup.EAhat / (2.0 * L),
                x0=x0, xm1=x0.copy(), c=c)


def string_chain_rule(setup, theta, inst, g, h_rel=1e-6):
    """dL/dtheta of a string from the per-mode gradients of modal_grad."""
    T0h, EIh, L, d1, d3 = (float(v) for v in theta)
    lam, om = inst["lam"], inst["omega"]
    gw, gg = g["omega"], g["gamma"]
    dT0 = np.sum(gw * lam / (2 * om))
    dEI = np.sum(gw * lam ** 2 / (2 * om))
    dd1 = np.sum(gg)
    dd3 = np.sum(gg * lam)
    # length: lambda_k = (k pi / L)^2, d lambda_k / dL = -2 lambda_k / L, in
    # omega, gamma and (with kappa ~ 1/L) the force's scale L^-5
    dlam = -2.0 * lam / L
    dL = (np.sum(gw * (2 * EIh * lam + T0h) * dlam / (2 * om)) + np.sum(gg * d3 * dlam)
          - 5.0 * g["scale"] / L)
    eps = h_rel * L
    xp, cp = _string_excitation(setup, L + eps)
    xm, cm = _string_excitation(setup, L - eps)
    dL += np.sum((g["x0"] + g["xm1"]) * (xp - xm) / (2 * eps)) + np.sum(g["c"] * (cp - cm) / (2 * eps))
    return np.array([dT0, dEI, dL, dd1, dd3])


class StringFn(torch.autograd.Function):
    """y = simulate(theta) for a batch of string parameter vectors; backward
    through modal_grad and string_chain_rule."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, setup: StringSetup, n_steps: int, ckpt: int = 512):
        th = theta.detach().double().cpu().numpy().reshape(-1, 5)
        insts = [string_instance(setup, t) for t in th]
        sim = modal.Sim(insts, setup.fs, flags=modal.FLAG_GRAD)
        y = sim.run(n_steps).clone()
        ctx.save = (sim, insts, th, setup, n_steps, ckpt)
        return y

    @staticmethod
    def backward(ctx, gy):
        sim, insts, th, setup, n_steps, ckpt = ctx.save
        g = sim.grad(n_steps, gy.contiguous().float(), ckpt_every=ckpt)
        out = np.stack([string_chain_rule(setup, th[b], insts[b], {k: v[b] for k, v in g.items()})
                        for b in range(len(insts))])
        sim.close()
        return torch.tensor(out, dtype=torch.float64).reshape(-1, 5), None, None, None


def fit(target: torch.Tensor, theta0, setup, n_steps: int, iters: int = 100,
        lr: float = 0.05, tol: float = 0.1, loss_fn=mrstft_loss, callback=None, free=None):
    """Adam with a one-cycle cosine schedule on unconstrained parameters,
    batched over rows of theta0.  A row that reaches tol is frozen there;
    the loop stops when every row has.  ``free``: the indices of the
    parameters that are fitted (default all five); the others keep their
    values from theta0 (their gradients are dropped before each step).
    ``setup``: a PlateSetup (ModalFn) or a StringSetup (StringFn).
    Returns (theta [B,5] and losses [B] of each row's best iterate,
    iterations, loss history)."""
    fixed = np.ones(5, bool)
    fixed[list(range(5)) if free is None else list(free)] = False
    fixed_t = torch.from_numpy(fixed)
    string = isinstance(setup, StringSetup)
    Fn = StringFn if string else ModalFn
    bounds = setup.bounds if string else (0.3, 1.5)
    z = torch.tensor(np.stack([to_unconstrained(t, bounds) for t in np.atleast_2d(theta0)]),
                     dtype=torch.float64, requires_grad=True)
    B = z.shape[0]
    opt = torch.optim.Adam([z], lr=lr)
    hist = []
    tgt = target.reshape(-1, target.shape[-1])
    best_L = np.full(B, np.inf)
    best_th = from_unconstrained(z, bounds).detach().numpy().copy()
    frozen = np.zeros(B, bool)
    z_frozen = z.detach().clone()
    it = 0
    for it in range(iters):
        for gparam in opt.param_groups:
            gparam["lr"] = one_cycle_cosine(it, iters, lr)
        opt.zero_grad()
        theta = from_unconstrained(z, bounds)
        y = Fn.apply(theta, setup, n_steps)
        L = loss_fn(y, tgt.expand_as(y), reduce=False)
        Ln = L.detach().cpu().numpy()
        hist.append(Ln)
        better = Ln < best_L
        best_L[better] = Ln[better]
        best_th[better] = theta.detach().numpy()[better]
        if callback:
            callback(it, theta.detach(), L.detach())
        newly = (Ln < tol) & ~frozen
        z_frozen[torch.from_numpy(newly)] = z.detach()[torch.from_numpy(newly)]
        frozen |= newly
        if frozen.all():
            return best_th, best_L, it, hist
        L.sum().backward()
        if fixed.any():
            z.grad[:, fixed_t] = 0.0
        opt.step()
        with torch.no_grad():  # frozen rows stay where they reached tol
            fz = torch.from_numpy(frozen)
            z[fz] = z_frozen[fz]
    return best_th, best_L, iters, hist


def symmetric_part(G: torch.Tensor) -> torch.Tensor:
    """(G + G^T) / 2 over the last two indices: the gradient with respect to a
    coupling tensor constrained, like the coupling coefficients, to be
    symmetric in its last two indices."""
    return 0.5 * (G + G.transpose(-1, -2))


def fit_tensor(inst: dict, target: torch.Tensor, H0, n_steps: int, iters: int = 100,
               lr: float = 0.05, loss_fn=mrstft_loss, ckpt: int = 512, fs: float = 44100.0,
               h_scale: float | None = None, callback=None):
    """Fits the coupling tensor of a von Karman instance, everything else
    fixed, to a target output (paper: Sec. 4.3, the coupling coefficients H
    optimised from a random normal start to match the displacement at a fixed
    point over 17 640 steps, with several starts explored in parallel).

    H0: one start [n_in, n_t, n_t] or B starts [B, n_in, n_t, n_t], each
    symmetric in its last two indices; the starts run as one batch.  Each
    iteration replaces the tensors (modal_set_tensor), runs the forward pass,
    takes dL/dy of loss_fn(y_b, target) per start by torch autograd, and runs
    modal_grad with the full tensor gradient; Adam steps on its symmetric
    part, which keeps every H exactly symmetric.  lr is relative to h_scale
    (default: the rms entry of H0); the schedule is the one-cycle cosine of
    the parameter fits.
    Returns (best H per start as a CUDA tensor shaped like H0, best loss per
    start [B], loss history [iterations][B])."""
    H0 = np.asarray(H0, np.float32)
    single = H0.ndim == 3
    H0 = H0[None] if single else H0
    B = H0.shape[0]
    H = torch.tensor(H0, device="cuda", requires_grad=True)
    # each start on one workgroup whose waves share its rows: a small plate's
    # step is latency-bound, and a slab exchange between workgroups costs more
    # than it saves
    sim = modal.Sim([dict(inst, Ht=H0[b]) for b in range(B)], fs, flags=modal.FLAG_GRAD)
    rms = float(H.detach().pow(2).mean().sqrt()) if h_scale is None else float(h_scale)
    opt = torch.optim.Adam([H], lr=lr * rms)
    tgt = target.reshape(1, -1).to(H.device)
    hist = []
    best_L = np.full(B, np.inf)
    best_H = H.detach().clone()
    try:
        for it in range(iters):
            for gparam in opt.param_groups:
                gparam["lr"] = one_cycle_cosine(it, iters, lr * rms)
            for b in range(B):
                sim.set_tensor(b, H.detach()[b])
            sim.reset()
            y = sim.run(n_steps).clone().requires_grad_(True)
            Ls = torch.stack([loss_fn(y[b:b + 1], tgt) for b in range(B)])
            Ls.sum().backward()
            Ln = Ls.detach().cpu().numpy()
            hist.append(Ln)
            better = Ln < best_L
            best_L[better] = Ln[better]
            best_H[torch.from_numpy(better).to(H.device)] = H.detach()[torch.from_numpy(better).to(H.device)]
            if callback:
                callback(it, Ln)
            g = sim.grad(n_steps, y.grad.float().contiguous(), ckpt_every=ckpt, tensor=True)
            H.grad = symmetric_part(torch.stack(g["H"]))
            opt.step()
            opt.zero_grad(set_to_none=True)
    finally:
        sim.close()
    if single:
        return best_H[0], float(best_L[0]), [float(h[0]) for h in hist]
    return best_H, best_L, hist
