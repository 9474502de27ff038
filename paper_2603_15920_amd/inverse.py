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


def inlet_pressure_observer(mesh, patch="inlet", device="cuda:0", with_capacitors=False):
    """obs(U, p, pc): the mean pressure over the cells next to a patch, followed by the Windkessel
    capacitor pressures when with_capacitors (a differentiable torch vector)."""
    pt = mesh.patch(patch)
    cells = torch.as_tensor(sorted(set(mesh.owner[pt.start:pt.start + pt.size].tolist())), device=device)

    def obs(U, p, pc):
        v = p[cells].mean().reshape(1)
        return torch.cat([v, pc.to(v.device)]) if with_capacitors else v
    return obs


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
