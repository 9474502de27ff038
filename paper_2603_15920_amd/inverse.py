"""Parameter inference through the differentiable PISO window (the paper's inverse problems, Sec. 3.3
and 3.4: gradient-based recovery of boundary parameters from time series of an observed quantity,
with the parameters optimised in log space so they stay positive).

A run is a chain of checkpointed windows (autograd.piso_window); after each window an observation
function of the state is recorded, and the loss is the mean squared misfit of the recorded series
against a target series.  torch.autograd composes the windows' discrete adjoints; the optimiser is
torch.optim.Adam on the log-parameters.  Marshalling only: every PISO step and adjoint step runs in
libdifvm.
"""
import torch

from .autograd import piso_window


def patch_pressure_observer(mesh, patches, device="cuda:0", with_capacitors=False):
    """obs(U, p, pc): the mean pressure over the cells next to each named patch, in the given order,
    followed by the Windkessel capacitor pressures when with_capacitors (a differentiable torch
    vector).  Next to an RCR outlet the pressure is about pc + Rp Q (eq. windkessel_Q), so observing
    the outlets as well as the capacitors makes the proximal resistances identifiable."""
    groups = []
    for name in patches:
        pt = mesh.patch(name)
        groups.append(torch.as_tensor(sorted(set(mesh.owner[pt.start:pt.start + pt.size].tolist())), device=device))

    def obs(U, p, pc):
        v = torch.stack([p[c].mean() for c in groups])
        return torch.cat([v, pc.to(v.device)]) if with_capacitors else v
    return obs


def inlet_pressure_observer(mesh, patch="inlet", device="cuda:0", with_capacitors=False):
    """obs(U, p, pc): the mean pressure over the cells next to a patch, followed by the Windkessel
    capacitor pressures when with_capacitors (a differentiable torch vector)."""
    return patch_pressure_observer(mesh, (patch,), device, with_capacitors)


def simulate_series(piso, theta, state0, n_windows, steps, observe, ckpt_every=None, adj_tol=1e-10):
    """Runs n_windows windows of `steps` steps from state0 = (U, p, phi, pc) with Windkessel parameters
    theta[n_wk, 3]; returns the stacked observations [n_windows, ...] (differentiable in theta and
    state0)."""
    U, p, phi, pc = state0
    obs = []
    for _ in range(n_windows):
        U, p, phi, pc = piso_window(piso, theta, U, p, phi, pc, steps, ckpt_every or steps, adj_tol)
        obs.append(observe(U, p, pc))
    return torch.stack(obs)


def fit_windkessel(piso, theta0, state0, target, n_windows, steps, observe, iters=20, lr=0.05, adj_tol=1e-10,
                   callback=None):
    """Adam on log(theta) to fit the observation series to `target`.  Returns (theta, history) with
    history a list of (loss, theta) per iteration, the loss being the mean squared misfit relative to
    the target's magnitude per observable."""
    log_theta = torch.log(torch.as_tensor(theta0, dtype=torch.float64)).clone().requires_grad_(True)
    opt = torch.optim.Adam([log_theta], lr=lr)
    target = torch.as_tensor(target, dtype=torch.float64, device=state0[0].device)
    history = []
    for it in range(iters):
        opt.zero_grad()
        theta = torch.exp(log_theta)
        series = simulate_series(piso, theta, state0, n_windows, steps, observe, adj_tol=adj_tol)
        scale = target.abs().mean(dim=0).clamp_min(1e-30)
        loss = (((series - target) / scale) ** 2).mean()
        loss.backward()
        history.append((float(loss.detach()), theta.detach().clone()))
        if callback:
            callback(it, history[-1])
        opt.step()
    return torch.exp(log_theta).detach(), history


def fit_boundary_scale(piso, pattern, s0, state0, probes, target, steps, iters=30, lr=0.1, betas=(0.7, 0.999),
                       ckpt_every=10, adj_tol=1e-10, callback=None):
    """Recovers a scalar s that scales a fixed velocity boundary pattern, U_b = s * pattern [Fb, 3] (the
    lid-velocity problem of Sec. 3.3.1: U_lid = (s, 0, 0) on the lid faces), from velocities probed at
    cells `probes` after `steps` steps from state0 = (U, p, phi, pc): Adam on s itself, the loss the
    mean squared misfit of the probed velocity components against `target` [n_probes, 3].  The initial
    flux state0[2] is an independent input held fixed (for a lid the boundary flux U_b . S is zero
    whatever s).  The first-moment decay 0.7 (torch's default is 0.9) damps the slow oscillation
    of a single parameter about its optimum.  Returns (s, history) with history (loss, s) per
    iteration."""
    s = torch.tensor(float(s0), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([s], lr=lr, betas=betas)
    U0, p0, phi0, pc0 = state0
    dev = U0.device
    pattern = torch.as_tensor(pattern, dtype=torch.float64, device=dev)
    target = torch.as_tensor(target, dtype=torch.float64, device=dev)
    probes = torch.as_tensor(probes, device=dev)
    theta = torch.zeros((0, 3), dtype=torch.float64)
    history = []
    for it in range(iters):
        opt.zero_grad()
        Ub = s.to(dev) * pattern
        U, p, phi_n, pc = piso_window(piso, theta, U0, p0, phi0, pc0, steps, ckpt_every, adj_tol, Ub=Ub)
        loss = ((U[probes] - target) ** 2).mean()
        loss.backward()
        history.append((float(loss.detach()), float(s.detach())))
        if callback:
            callback(it, history[-1])
        opt.step()
    return float(s.detach()), history
