"""torch.autograd.Function over the checkpointed PISO window.

PisoWindow.apply(theta, U0, p0, phi0, pc0, Ub, piso, nsteps, ckpt_every, adj_tol) runs nsteps PISO
steps through difvm_piso_forward_record and returns (U_N, p_N, phi_N, pc_N); its backward calls
difvm_piso_adjoint (the library's discrete adjoint) and returns gradients for the Windkessel
parameters theta[n_wk, 3] = (Rp, C, Rd) per outlet, for the initial state and, when Ub (the fixed
velocity boundary values [Fb, 3], or None to keep the PISO's) is given, for Ub
(difvm_tape_boundary_cotangent).  All arrays are in user order; U0, p0, phi0, Ub are float64 tensors
on the context's device, theta and pc0 float64 tensors (any device).  Marshalling only: the
computation is in libdifvm.
"""
import numpy as np
import torch

from . import binding as B


class PisoWindow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, U0, p0, phi0, pc0, Ub, piso, nsteps, ckpt_every, adj_tol):
        n_wk = piso.mesh.info["n_windkessel"]
        if Ub is not None:
            piso.set_boundary(Ub.detach().contiguous(), None)
        th = theta.detach().double().cpu().numpy().reshape(-1, 3) if n_wk else np.zeros((0, 3))
        pcv = pc0.detach().double().cpu().numpy().reshape(-1) if n_wk else np.zeros(0)
        for j in range(n_wk):
            piso.set_windkessel(j, th[j, 0], th[j, 1], th[j, 2], pcv[j])
        piso.set_state(U0.detach().contiguous(), p0.detach().contiguous(), phi0.detach().contiguous())
        ctx.tape = None
        if not any(ctx.needs_input_grad[:6]):
            # nothing to differentiate: plain steps, no tape (the same arithmetic)
            status, iters, _ = piso.step(nsteps)
            U, p, phi, pc = piso.get_state()
            ctx.status, ctx.iters = status, iters
            return U, p, phi, torch.as_tensor(pc, dtype=torch.float64, device=pc0.device)
        tape = B.difvm_tape_create(piso.h, nsteps, ckpt_every)
        try:
            status, iters = B.difvm_piso_forward_record(piso.h, tape, nsteps, piso.params.n_corr)
        except Exception:
            B.difvm_tape_destroy(tape)
            raise
        U, p, phi, pc = piso.get_state()
        ctx.piso, ctx.tape, ctx.adj_tol, ctx.n_wk = piso, tape, adj_tol, n_wk
        ctx.theta_dev, ctx.pc_dev = theta.device, pc0.device
        ctx.status, ctx.iters = status, iters
        return U, p, phi, torch.as_tensor(pc, dtype=torch.float64, device=pc0.device)

    @staticmethod
    def backward(ctx, gU, gp, gphi, gpc):
        if ctx.tape is None:
            raise RuntimeError("PisoWindow: this window was run without a tape (no input required grad)")
        piso, n_wk = ctx.piso, ctx.n_wk
        src = piso.mesh.src
        dev = piso.mesh.ctx.device
        gU0 = torch.empty((src.n_cells, 3), dtype=torch.float64, device=dev)
        gp0 = torch.empty(src.n_cells, dtype=torch.float64, device=dev)
        gphi0 = torch.empty(src.n_faces, dtype=torch.float64, device=dev)
        gpc_np = None if gpc is None else gpc.detach().double().cpu().numpy().reshape(-1)
        cont = lambda t: None if t is None else t.detach().double().contiguous()
        gUb = None
        try:
            _, gpc0, gwk = B.difvm_piso_adjoint(piso.h, ctx.tape, cont(gU), cont(gp), cont(gphi), gpc_np, ctx.adj_tol,
                                                gU0, gp0, gphi0, n_wk)
            if ctx.needs_input_grad[5]:
                gUb = torch.empty((src.n_boundary_faces, 3), dtype=torch.float64, device=dev)
                B.difvm_tape_boundary_cotangent(ctx.tape, gUb)
        finally:
            B.difvm_tape_destroy(ctx.tape)
            ctx.tape = None
        gtheta = torch.as_tensor(gwk, dtype=torch.float64, device=ctx.theta_dev)
        gpc0 = torch.as_tensor(gpc0, dtype=torch.float64, device=ctx.pc_dev)
        return gtheta, gU0, gp0, gphi0, gpc0, gUb, None, None, None, None


def piso_window(piso, theta, U0, p0, phi0, pc0, nsteps, ckpt_every=10, adj_tol=1e-10, Ub=None):
    """Differentiable N-step PISO window; returns (U_N, p_N, phi_N, pc_N).  Ub: fixed velocity boundary
    values [Fb, 3] to differentiate (None keeps the values set on the PISO)."""
    return PisoWindow.apply(theta, U0, p0, phi0, pc0, Ub, piso, int(nsteps), int(ckpt_every), float(adj_tol))
