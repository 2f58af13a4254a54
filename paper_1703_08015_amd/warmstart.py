"""Learned warm start: steady states from the batched solver train the U-Net,
whose (rho, u) prediction initialises the solver through f_eq (lbm_init).

The prediction is first given the invariants of a start from rest
(lbm_project_invariants): mass rho0 per node on every lattice-connected
component, and a momentum field with no component along any of the step's
staggered invariants (a few sweeps of the link operator).  The discrete
dynamics never change those, so without the projection a warm start settles
into a different long-time state than the cold start.

The solver still produces the answer: a warm run steps to the same residual
tolerance as a cold start from rest, and falls back to a cold start if its
residual turns non-finite or grows.
"""
import time

import numpy as np

from . import lbm, nn
from .unet import UNet


def nu_of(tau):
    return (tau - 0.5) / 3.0


class Sample:
    """One geometry on the GPU: mask, force, and (after the solver) its
    steady fields, channels last."""

    def __init__(self, torch, mask, g, rho=None, u=None):
        self.shape = tuple(mask.shape)
        self.g = np.asarray(g, np.float64)
        self.gmag = float(np.linalg.norm(self.g))
        self.dir = self.g / self.gmag
        self.solid = torch.from_numpy(np.ascontiguousarray(mask.astype(np.uint8))).cuda()
        self.rho, self.u = rho, u  # torch FP64 (nz,ny,nx) and (3,nz,ny,nx)
        self.target = None
        self.x = None  # cached network input (encode)
        self.energy = None  # sum of squared targets (train)
        self._mask = np.asarray(mask, bool)
        self._inv = None

    @property
    def invariants(self):
        """Component labels of the geometry, computed on the GPU from the
        device mask (lbm_components_device) on first use."""
        if self._inv is None:
            self._inv = lbm.Invariants(self.solid, 19)
        return self._inv


def steady_dataset(torch, masks, gs, tau=0.8, storage="f32", tol=1e-6, check_every=100, max_steps=200000,
                   progress=None):
    """Run all geometries as one batch to steady state; return Samples with
    rho, u and the number of steps each needed."""
    tiles = lbm.Tiles.concat([lbm.Tiles(m) for m in masks])
    s = lbm.Solver(tiles, lattice=19, storage=storage, tau=tau, persistent=1, graph_steps=check_every)
    s.set_sample_force(np.asarray(gs, np.float64))
    s.init()
    steps, res = s.run_to_steady(tol=tol, check_every=check_every, max_steps=max_steps, progress=progress)
    rho, u = s.moments()
    out = []
    o = 0
    for m, g in zip(masks, gs):
        n = m.size
        r = rho[o:o + n].view(m.shape)
        uu = u[3 * o:3 * (o + n)].view((3,) + m.shape)
        out.append(Sample(torch, m, g, r.clone(), uu.clone()))
        o += n
    del s
    return out, steps, res


def training_view(torch, sample, multiple=8):
    """The sample as the network trains on it: every edge must be a multiple
    of 2^(levels-1) = 8.  A periodic cube whose edge is not is tiled twice
    along each axis; the doubled box is periodic too and, since the discrete
    step commutes with translations, its steady state from rest is exactly
    the tiled steady state, so geometry and target stay consistent."""
    if all(n % multiple == 0 for n in sample.shape):
        return sample
    if any((2 * n) % multiple for n in sample.shape):
        raise ValueError("edges %s cannot be doubled to multiples of %d" % (sample.shape, multiple))
    mask = np.tile(sample._mask, (2, 2, 2))
    rho = sample.rho.repeat(2, 2, 2)
    u = sample.u.repeat(1, 2, 2, 2)
    return Sample(torch, mask, sample.g, rho, u)


def make_targets(torch, samples, tau, rho0=1.0, out_scale=None):
    """Scaled targets (rho - rho0, u) * nu / |g| / out_scale as FP32
    (nz, ny, nx, 4); out_scale defaults to the RMS of the scaled velocity."""
    nu = nu_of(tau)
    if out_scale is None:
        acc, cnt = 0.0, 0
        for sm in samples:
            fl = sm.solid == 0
            uu = sm.u[:, fl] * (nu / sm.gmag)
            acc += float((uu ** 2).sum())
            cnt += int(uu.numel())
        out_scale = float(np.sqrt(acc / max(cnt, 1)))
    for sm in samples:
        k = nu / sm.gmag / out_scale
        t = torch.empty(sm.shape + (4,), dtype=torch.float32, device="cuda")
        t[..., 0] = ((sm.rho - rho0) * k).float()
        t[..., 1:] = (sm.u * k).permute(1, 2, 3, 0).float()
        t[sm.solid != 0] = 0.0
        sm.target = t
    return out_scale


# geometry input: link-path distance d to the nearest solid node, fed as
# s = min(d / 8, 4) and s^2 (slow flow in a pore grows with the square of the
# distance to its walls)
DIST_SCALE, DIST_CAP, DIST_SWEEPS = 0.125, 4.0, 64


def encode(torch, sample):
    """Geometry-only input (solid flag, distance to solid and its square),
    computed on the GPU and cached on the sample; the force direction enters
    through the force-linear output head."""
    if getattr(sample, "x", None) is None:
        d = torch.empty(sample.shape, dtype=torch.float32, device="cuda")
        tmp = torch.empty_like(d)
        nn.distance(sample.solid, d, tmp, DIST_SWEEPS, periodic=7)
        x = torch.empty(sample.shape + (8,), dtype=torch.bfloat16, device="cuda")
        nn.encode_geometry(sample.solid, d, DIST_SCALE, DIST_CAP, x)
        sample.x = x
    return sample.x


def make_net(levels=4, base=24, seed=0, out_scale=1.0):
    return UNet(levels=levels, base=base, out_ch=12, seed=seed, out_scale=out_scale)


def _energy(torch, sm):
    """Sum of the squared targets over fluid nodes (the loss of a zero
    prediction), computed once per sample with the library's MSE kernel."""
    if getattr(sm, "energy", None) is None:
        zero = torch.zeros(sm.shape + (4,), dtype=torch.float32, device="cuda")
        acc = torch.zeros(1, dtype=torch.float32, device="cuda")
        scratch = torch.empty(sm.shape + (8,), dtype=torch.bfloat16, device="cuda")
        nn.mse(zero[..., 0].numel(), 4, zero, sm.target, sm.solid, 1.0, scratch, 8, acc)
        sm.energy = max(float(acc.item()), 1e-30)
    return sm.energy


def train(torch, net, samples, epochs=10, lr=1e-3, seed=0, progress=None, lr_final=None):
    """Per-sample Adam steps on the masked squared error relative to the
    sample's own target energy (slow-flow magnitudes span orders of magnitude
    across porosities and grain sizes, and an absolute MSE would learn only
    the most permeable samples), learning rate decaying from lr to lr_final
    (default lr / 10) on a cosine.  Returns the mean relative squared error
    per epoch."""
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    history = []
    lr_final = lr / 10.0 if lr_final is None else lr_final
    for ep in range(epochs):
        frac = ep / max(epochs - 1, 1)
        lr_ep = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
        total = 0.0
        for idx in rng.permutation(len(samples)):
            sm = samples[idx]
            x = encode(torch, sm)
            energy = _energy(torch, sm)
            pred = net.forward_mixed(x, sm.dir)
            dout = torch.empty(sm.shape + (8,), dtype=torch.bfloat16, device="cuda")
            loss.zero_()
            nn.mse(pred[..., 0].numel(), 4, pred, sm.target, sm.solid, 1.0 / energy, dout, 8, loss)
            net.zero_grad()
            net.backward_mixed(dout, 8, sm.dir)
            net.adam_step(lr_ep)
            total += float(loss.item()) / energy  # the kernel accumulates the unscaled sum
        history.append(total / max(len(samples), 1))
        if progress:
            progress(ep, history[-1])
    return history


def predict_fields(torch, net, sample, tau, rho0=1.0, project=True):
    """Network (rho, u) for a geometry as dense FP64 fields, projected onto
    the invariants of a start from rest (project=False: the raw decode)."""
    x = encode(torch, sample)
    pred = net.forward_mixed(x, sample.dir)
    rho = torch.empty(sample.shape, dtype=torch.float64, device="cuda")
    u = torch.empty((3,) + sample.shape, dtype=torch.float64, device="cuda")
    nn.decode_output(pred, sample.solid, rho0, net.out_scale * sample.gmag / nu_of(tau), rho, u, renorm=False)
    if project:
        sample.invariants.project(rho, u, rho0)
    return rho, u


def solve(torch, sample, tau, init=None, storage="f32", tol=1e-6, check_every=100, max_steps=200000,
          with_rho=False):
    """Run one geometry to steady state from rest (init None) or from given
    (rho, u); returns (steps, seconds, final u, fell_back), and the final rho
    after them if with_rho."""
    tiles = lbm.Tiles(sample.solid.cpu().numpy().astype(bool))
    s = lbm.Solver(tiles, lattice=19, storage=storage, tau=tau, g=tuple(sample.g), graph_steps=check_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fell_back = False
    if init is None:
        s.init()
    else:
        s.init(*init)
        # guard: a prediction whose first residuals are non-finite or growing falls back to rest
        s.step(check_every)
        try:
            r1 = s.residual()[0]
            s.step(check_every)
            r2 = s.residual()[0]
            bad = not (np.isfinite(r1) and np.isfinite(r2)) or r2 > 2.0 * r1
        except lbm.LbmError:
            bad = True
        if bad:
            fell_back = True
            s.init()
    steps, res = s.run_to_steady(tol=tol, check_every=check_every, max_steps=max_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rho, u = s.moments()
    taken = int(s.step_count)
    del s
    out = (taken if steps[0] > 0 else -1, wall, u, fell_back)
    return out + (rho,) if with_rho else out


def evaluate(torch, net, samples, tau, storage="f32", tol=1e-6, check_every=100, project=True, fp64_cold=False):
    """Warm vs cold time to steady state for each geometry (project=False
    starts from the raw prediction, for comparison; fp64_cold also times the
    plain FP64 solver from rest and checks the warm answer against it)."""
    rows = []
    for sm in samples:
        cold_steps, cold_s, u_cold, _ = solve(torch, sm, tau, None, storage, tol, check_every)
        extra = {}
        if fp64_cold:
            s64, t64, u64, _ = solve(torch, sm, tau, None, "f64", tol, check_every)
            extra = dict(cold_f64_steps=s64, cold_f64_s=t64, u64=u64)
        # everything only the warm path needs is timed with it: the geometry
        # input, the forward pass, the component labels (on the GPU) and the
        # projection; the tiling, which both paths need, is timed by neither
        sm.x = None
        sm._inv = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if project:
            sm.invariants
        torch.cuda.synchronize()
        t_lab = time.perf_counter() - t0
        init = predict_fields(torch, net, sm, tau, project=project)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        fl = sm.solid == 0
        up, uc = init[1][:, fl], u_cold[:, fl]
        norm = float((uc ** 2).sum().sqrt())
        pred_err = float(((up - uc) ** 2).sum().sqrt()) / norm
        # the same error after the best single scale factor on the prediction:
        # how much of it is the overall magnitude rather than the shape
        alpha = float((up * uc).sum() / (up * up).sum().clamp_min(1e-300))
        pred_err_scaled = float(((alpha * up - uc) ** 2).sum().sqrt()) / norm
        warm_steps, warm_s, u_warm, fb = solve(torch, sm, tau, init, storage, tol, check_every)
        agree = float(((u_warm[:, fl] - u_cold[:, fl]) ** 2).sum().sqrt() / (u_cold[:, fl] ** 2).sum().sqrt())
        row = dict(cold_steps=cold_steps, cold_s=cold_s, warm_steps=warm_steps, warm_s=warm_s + t_inf,
                   inference_s=t_inf, labels_s=t_lab, solve_s=warm_s, prediction_u_rel_l2=pred_err,
                   prediction_best_scale=alpha, prediction_u_rel_l2_best_scale=pred_err_scaled,
                   warm_vs_cold_u_rel_l2=agree, fell_back=fb)
        if extra:
            u64 = extra.pop("u64")
            row.update(extra)
            row["warm_vs_cold_f64_u_rel_l2"] = float(((u_warm[:, fl] - u64[:, fl]) ** 2).sum().sqrt() /
                                                     (u64[:, fl] ** 2).sum().sqrt())
        rows.append(row)
    return rows


def error_curve(torch, net, sample, tau, scales=(0.0, 0.03, 0.1, 0.3, 1.0), storage="f32", tol=1e-6,
                check_every=100):
    """Steps to steady state against the error of the starting fields.  The
    exact steady fields (rho*, u*) of a cold run are moved towards the
    network's prediction, (rho*, u*) + s (prediction - (rho*, u*)) for each
    scale s, projected onto the invariants of rest and solved from there:
    s = 1 is the network itself, s = 0 the best any f_eq start can do.
    Returns the cold run and one row per scale."""
    cold_steps, cold_s, u_ref, _, rho_ref = solve(torch, sample, tau, None, storage, tol, check_every,
                                                  with_rho=True)
    rho_p, u_p = predict_fields(torch, net, sample, tau, project=False)
    fl = sample.solid == 0
    norm = float((u_ref[:, fl] ** 2).sum().sqrt())
    rows = []
    for sc in scales:
        rho = rho_ref + sc * (rho_p - rho_ref)
        u = u_ref + sc * (u_p - u_ref)
        err = float(((u - u_ref)[:, fl] ** 2).sum().sqrt()) / norm
        sample.invariants.project(rho, u, 1.0)
        steps, secs, _, fb = solve(torch, sample, tau, (rho, u), storage, tol, check_every)
        rows.append(dict(scale=sc, start_u_rel_l2=err, steps=steps, seconds=secs, fell_back=fb))
    return dict(cold_steps=cold_steps, cold_s=cold_s), rows
