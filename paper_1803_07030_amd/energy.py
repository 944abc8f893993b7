"""Energy of Eq. 1 (paper, section "Classical spin Hamiltonian") as a
differentiable function of the spins, the per-bond exchange constants, the
per-site anisotropy constants and the field intensity, with the forward and
the vector-Jacobian product computed by the library's HIP kernels
(hsim_energy_forward / hsim_energy_backward), and the fluctuation estimator of
derivatives of thermal averages (hsim_fluct_estimate)."""
import torch

from . import hsim


def _check_inputs(spins, J_bond, k, axis, field_dir, plan):
    """The kernels read raw pointers of the spins' precision: every tensor
    must have the spins' dtype and shape, and live on the spins' GPU."""
    if not isinstance(spins, torch.Tensor) or spins.dtype not in (torch.float32, torch.float64):
        raise TypeError("spins must be a float32 or float64 tensor [batch, 3, n]")
    n, nb = int(plan.n), int(plan.info.n_bonds)
    if spins.dim() != 3 or spins.shape[1] != 3 or spins.shape[2] != n:
        raise ValueError(f"spins must have shape [batch, 3, {n}], got {tuple(spins.shape)}")
    want = {"J_bond": (J_bond, (nb,)), "k": (k, (n,)), "axis": (axis, (3, n))}
    if field_dir is not None:
        want["field_dir"] = (field_dir, (3, n))
    for name, (t, shape) in want.items():
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a tensor")
        if t.dtype != spins.dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, the spins {spins.dtype}: "
                            "every input must have the spins' precision")
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {list(shape)}, got {list(t.shape)}")
    for name, t in [("spins", spins)] + [(nm, v[0]) for nm, v in want.items()]:
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be on a CUDA device, got {t.device}")
        if t.device != spins.device:
            raise ValueError(f"{name} is on {t.device}, the spins on {spins.device}")


class HeisenbergEnergy(torch.autograd.Function):
    """E_b(S_b; J, k, B) for a batch of configurations S [batch, 3, n] (user
    order) on one plan; J per bond in the plan's bond order, k [n], axis
    [3, n], B a 0-d tensor, field_dir [3, n] or None (+z).  float32 inputs use
    the FP32 kernels with double accumulation, float64 inputs the FP64 ones.
    Returns E [batch] in float64."""

    @staticmethod
    def forward(ctx, spins, J_bond, k, B, plan, axis, field_dir):
        _check_inputs(spins, J_bond, k, axis, field_dir, plan)
        prec = hsim.FP64_EXACT if spins.dtype == torch.float64 else hsim.FP32
        spins = spins.contiguous()
        J_bond, k, axis = J_bond.contiguous(), k.contiguous(), axis.contiguous()
        fd = None if field_dir is None else field_dir.contiguous()
        batch = spins.shape[0]
        E = torch.empty(batch, dtype=torch.float64, device=spins.device)
        hsim.hsim_energy_forward(plan.handle, batch, prec, spins, J_bond, k, axis, float(B), fd, E)
        ctx.save_for_backward(spins, J_bond, k, axis)
        ctx.fd, ctx.plan, ctx.prec, ctx.B = fd, plan, prec, float(B)
        return E

    @staticmethod
    def backward(ctx, gE):
        spins, J_bond, k, axis = ctx.saved_tensors
        gE = gE.contiguous().to(torch.float64)
        batch = spins.shape[0]
        need = ctx.needs_input_grad
        gS = torch.empty_like(spins) if need[0] else None
        gJ = torch.empty_like(J_bond) if need[1] else None
        gk = torch.empty_like(k) if need[2] else None
        gB = torch.empty(1, dtype=torch.float64, device=spins.device) if need[3] else None
        hsim.hsim_energy_backward(ctx.plan.handle, batch, ctx.prec, spins, J_bond, k, axis, ctx.B,
                                  ctx.fd, gE, gS, gJ, gk, gB)
        gBt = None if gB is None else gB.reshape(())
        return gS, gJ, gk, gBt, None, None, None


def heisenberg_energy(spins, J_bond, k, B, plan, axis, field_dir=None):
    return HeisenbergEnergy.apply(spins, J_bond, k, B, plan, axis, field_dir)


def fluct_estimate(beta, O, dE, dO=None):
    """d<O>/dtheta = <dO/dtheta> - beta Cov(O, dE/dtheta) over the samples
    (fluctuation-dissipation form of the derivative of a canonical average).
    Returns (estimate, covariance) as a float64 tensor of 2 elements."""
    for name, t in (("O", O), ("dE", dE), ("dO", dO)):
        if t is None:
            continue
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be on a CUDA device, got {t.device}")
        if t.numel() != O.numel():
            raise ValueError(f"{name} has {t.numel()} samples, O has {O.numel()}")
    O = O.contiguous().to(torch.float64)
    dE = dE.contiguous().to(torch.float64)
    dO = None if dO is None else dO.contiguous().to(torch.float64)
    out = torch.empty(2, dtype=torch.float64, device=O.device)
    hsim.hsim_fluct_estimate(O.numel(), beta, O, dE, dO, out)
    return out


def spins_planar(spins_site_major, dtype=torch.float64):
    """Site-major double spins [n_cfg, n, 3] (snapshots, spins_user) as the
    planar [n_cfg, 3, n] tensor of the energy calls, converted by the
    library's kernel."""
    s = spins_site_major
    if s.dtype != torch.float64 or s.dim() != 3 or s.shape[2] != 3 or s.device.type != "cuda":
        raise ValueError("spins must be a CUDA float64 tensor [n_cfg, n, 3]")
    s = s.contiguous()
    out = torch.empty((s.shape[0], 3, s.shape[1]), dtype=dtype, device=s.device)
    prec = hsim.FP64_EXACT if dtype == torch.float64 else hsim.FP32
    hsim.hsim_spins_planar(s.shape[0], s.shape[1], s, prec, out)
    return out


def fluct_gradients(plan, spins, J_bond, k, axis, B, beta, field_dir=None, O=None):
    """Fluctuation estimate of d<O>/dJ_bond, d<O>/dk and d<O>/dB from
    configurations spins [n_cfg, 3, n] sampled at inverse temperature beta:
    d<O>/dtheta = <dO/dtheta> - beta Cov(O, dE/dtheta).  O [n_cfg] float64
    (device) is an observable that does not depend on the parameters, or None
    for the energy itself.  One forward (for O = E), one weight kernel and one
    backward, all in the library.  Returns (gJ, gk, gB, O)."""
    _check_inputs(spins, J_bond, k, axis, field_dir, plan)
    prec = hsim.FP64_EXACT if spins.dtype == torch.float64 else hsim.FP32
    spins, J_bond, k, axis = spins.contiguous(), J_bond.contiguous(), k.contiguous(), axis.contiguous()
    fd = None if field_dir is None else field_dir.contiguous()
    n_cfg = spins.shape[0]
    c = 0.0
    if O is None:
        O = torch.empty(n_cfg, dtype=torch.float64, device=spins.device)
        hsim.hsim_energy_forward(plan.handle, n_cfg, prec, spins, J_bond, k, axis, float(B), fd, O)
        c = 1.0
    elif O.dtype != torch.float64 or O.numel() != n_cfg or O.device != spins.device:
        raise ValueError(f"O must be a float64 tensor of {n_cfg} samples on {spins.device}")
    O = O.contiguous()
    w = torch.empty(n_cfg, dtype=torch.float64, device=spins.device)
    hsim.hsim_fluct_weights(n_cfg, beta, O, c, w)
    gJ, gk = torch.empty_like(J_bond), torch.empty_like(k)
    gB = torch.empty(1, dtype=torch.float64, device=spins.device)
    hsim.hsim_energy_backward(plan.handle, n_cfg, prec, spins, J_bond, k, axis, float(B), fd, w,
                              None, gJ, gk, gB)
    return gJ, gk, gB, O
