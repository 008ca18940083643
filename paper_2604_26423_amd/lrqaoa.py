"""LR-QAOA on top of libqs: schedule, angle conventions, a simulator object and
a torch.autograd.Function for the adjoint gradient.

arXiv:2604.26423, Sec. II-B: p layers of the cost unitary exp(-i gamma_k H_C)
(eq. 2) and the mixer exp(+i beta_k H_B) (eq. 3) on |+>^n, with the linear
ramp of eq. (4).  libqs works in gate angles -- RZZ(theta_zz w_ij) on every
pair and RX(theta_x) on every qubit -- so this module only maps angles; all
state arithmetic runs in the HIP library.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import qs as _qs

PRECISIONS = {"c64": _qs.QS_C64, "c128": _qs.QS_C128}


# ---------------------------------------------------------------- schedule
def linear_ramp(p: int, delta_gamma: float, delta_beta: float, form: str = "midpoint"):
    """Per-layer (gamma_k, beta_k).

    form="paper": eq. (4), gamma_i = (i+1)/p D_gamma, beta_i = (1 - i/p) D_beta, i = 0..p-1.
    form="midpoint": gamma_k = (k - 1/2)/p D_gamma, beta_k = (1 - (k - 1/2)/p) D_beta, k = 1..p.
    """
    if form == "paper":
        frac_g = [(i + 1) / p for i in range(p)]
        frac_b = [1 - i / p for i in range(p)]
    elif form == "midpoint":
        frac_g = [(k - 0.5) / p for k in range(1, p + 1)]
        frac_b = [1 - (k - 0.5) / p for k in range(1, p + 1)]
    else:
        raise ValueError(form)
    return (np.array([f * delta_gamma for f in frac_g]), np.array([f * delta_beta for f in frac_b]))


def ramp_weights(p: int, form: str = "midpoint"):
    """d gamma_k / d D_gamma and d beta_k / d D_beta of linear_ramp."""
    g, b = linear_ramp(p, 1.0, 1.0, form)
    return g, b


# Gate-angle conventions.  "paper": exp(-i gamma H_C) = prod RZZ(2 gamma w_ij),
# exp(+i beta sum X) = prod RX(-2 beta).  "literal": RZZ(gamma w_ij), RX(2 beta).
_CONV = {"paper": (2.0, -2.0), "literal": (1.0, 2.0)}


def to_gate_angles(gammas, betas, convention: str = "paper"):
    a, b = _CONV[convention]
    return a * np.asarray(gammas, dtype=np.float64), b * np.asarray(betas, dtype=np.float64)


def gate_grad_to_schedule(d_theta_zz, d_theta_x, convention: str = "paper"):
    """Chain rule: (dE/dgamma_k, dE/dbeta_k) from (dE/dtheta_zz, dE/dtheta_x)."""
    a, b = _CONV[convention]
    return a * np.asarray(d_theta_zz), b * np.asarray(d_theta_x)


def n_from_edges(m: int) -> int:
    n = int(round((1 + math.sqrt(1 + 8 * m)) / 2))
    if n * (n - 1) // 2 != m:
        raise ValueError(f"{m} weights is not n(n-1)/2 for any n")
    return n


# ---------------------------------------------------------------- simulator
def sym_z_to_x(z, n: int):
    """Full basis index y(z) (bit n-1 clear) of complement-symmetric index z:
    y_q = z_q XOR z_(q+1) XOR ... XOR z_(n-2) (a suffix XOR)."""
    y = np.asarray(z, dtype=np.uint64).copy()
    sh = 1
    while sh < 64:
        y ^= y >> np.uint64(sh)
        sh <<= 1
    return y


def sym_x_to_z(x, n: int):
    """Complement-symmetric index of basis state x (x and ~x share it)."""
    x = np.asarray(x, dtype=np.uint64)
    top = (x >> np.uint64(n - 1)) & np.uint64(1)
    full = np.uint64((1 << n) - 1)
    y = np.where(top == 1, x ^ full, x)
    return y ^ (y >> np.uint64(1))


class Simulator:
    """One LR-QAOA instance on one GPU: cost diagonal, state, readouts.

    Device memory (state, diagonal, optional adjoint vector) is held in torch
    tensors; the HIP stream is torch's current stream at construction.
    symmetric=True stores only the complement-symmetric half (2^(n-1)
    amplitudes in z order, see include/qs.h, QS_SYM): half the memory and
    traffic; results refer to the full state.
    """

    def __init__(self, w_tenths, precision: str = "c64", device: str = "cuda", stream=None,
                 symmetric: bool = False):
        import torch
        self.torch = torch
        self.w = np.ascontiguousarray(np.asarray(w_tenths, dtype=np.int32))
        self.n = n_from_edges(len(self.w))
        self.precision = precision
        self.prec = PRECISIONS[precision]
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cdt = torch.complex64 if self.prec == _qs.QS_C64 else torch.complex128
        self.symmetric = bool(symmetric)
        nst = self.n - 1 if self.symmetric else self.n
        self.psi = torch.empty(1 << nst, dtype=cdt, device=self.device)
        self.diag = torch.empty(1 << nst, dtype=torch.int32, device=self.device)
        self.lam: Optional[object] = None
        flags = self.prec | (_qs.QS_SYM if self.symmetric else 0)
        self.handle = _qs.qs_alloc(self.n, flags, self.psi, self.psi.numel() * self.psi.element_size(),
                                   self.stream)
        diag_fn = _qs.qs_cost_diagonal_sym if self.symmetric else _qs.qs_cost_diagonal
        self.w_total, self.cmax = diag_fn(self.n, self.w, self.diag, self.stream)

    # ---- circuit
    def forward(self, theta_zz, theta_x, readout: bool = True):
        return _qs.qs_forward(self.handle, self.diag, self.w_total, theta_zz, theta_x, readout)

    def forward_schedule(self, gammas, betas, convention: str = "paper", readout: bool = True):
        tzz, tx = to_gate_angles(gammas, betas, convention)
        return self.forward(tzz, tx, readout)

    def init_plus(self):
        _qs.qs_init_plus(self.handle)

    def apply_cost_layer(self, theta_zz: float):
        _qs.qs_apply_cost_layer(self.handle, self.diag, self.w_total, theta_zz)

    def apply_mixer(self, theta_x: float):
        _qs.qs_apply_mixer(self.handle, theta_x)

    # ---- readouts
    def expect(self):
        return _qs.qs_expect(self.handle, self.diag)

    def ratio(self, exp_c: float) -> float:
        """r = <C> / C(x*) (eq. 5 with exact probabilities)."""
        return exp_c / (self.cmax / 10.0)

    def sample(self, shots: int, seed: int, on_device: bool = False):
        if on_device:
            out = self.torch.empty(shots, dtype=self.torch.int64, device=self.device)
            return _qs.qs_sample(self.handle, seed, shots, out)
        return _qs.qs_sample(self.handle, seed, shots)

    def shots_ratio(self, shots) -> float:
        """r of eq. (5) from sampled bitstrings."""
        shots = np.asarray(shots, dtype=np.uint64)
        if self.symmetric:
            shots = sym_x_to_z(shots, self.n)
        idx = self.torch.as_tensor(_qs.layout_indices(shots.astype(np.int64)), device=self.device)
        cuts = self.diag[idx].double().mean().item() / 10.0
        return cuts / (self.cmax / 10.0)

    def cost_histogram(self, on_device: bool = False):
        """Fixed-point mass of every cut value 0..W_t (tenths); 2^62 = probability 1."""
        nb = int(self.w_total) + 1
        if on_device:
            out = self.torch.empty(nb, dtype=self.torch.int64, device=self.device)
            return _qs.qs_cost_histogram(self.handle, self.diag, nb, out)
        return _qs.qs_cost_histogram(self.handle, self.diag, nb)

    def ratio_distribution(self):
        """(r values, probabilities): the exact distribution of C(x)/C(x*) under
        the state, from the cut-value histogram."""
        mass = self.cost_histogram().astype(np.float64)
        cut = np.arange(len(mass), dtype=np.float64)
        return cut / self.cmax, mass / mass.sum()

    def adjoint(self, theta_zz, theta_x, mode: str = "uncompute"):
        """(E, dE/dtheta_zz, dE/dtheta_x).  mode "uncompute" undoes every pass on
        psi (two state vectors at any depth); "store" keeps the state after every
        tile pass in a checkpoint buffer (qs_adjoint_ckpt_bytes) and reads it back."""
        if self.lam is None:
            self.lam = self.torch.empty_like(self.psi)
        lb = self.lam.numel() * self.lam.element_size()
        if mode == "uncompute":
            return _qs.qs_adjoint_grad(self.handle, self.diag, self.w_total, theta_zz, theta_x, self.lam, lb)
        if mode != "store":
            raise ValueError(f"mode must be 'uncompute' or 'store', not {mode!r}")
        nb = _qs.qs_adjoint_ckpt_bytes(self.handle, len(np.atleast_1d(theta_zz)))
        ck = self.torch.empty(max(nb, 1), dtype=self.torch.uint8, device=self.device) if nb else None
        try:
            return _qs.qs_adjoint_grad_store(self.handle, self.diag, self.w_total, theta_zz, theta_x, ck, nb,
                                             self.lam, lb)
        finally:
            del ck

    def release_adjoint(self):
        self.lam = None

    def state(self):
        """The state buffer as stored (layout of qs_layout_index)."""
        return self.psi

    def amplitudes(self):
        """The stored amplitudes in index order (z order for the symmetric layout), a new device tensor."""
        out = self.torch.empty_like(self.psi)
        return _qs.qs_get_amplitudes(self.handle, 0, self.psi.numel(), out)

    def set_amplitudes(self, values):
        """Overwrite the stored amplitudes from a device tensor in index order."""
        _qs.qs_set_amplitudes(self.handle, 0, values.to(self.psi.dtype).contiguous())

    def diagonal(self):
        """The cost diagonal in index order (a read-back through the layout map)."""
        idx = self.torch.as_tensor(_qs.layout_indices(np.arange(self.diag.numel(), dtype=np.int64)),
                                   device=self.device)
        return self.diag[idx]

    def full_state(self):
        """The state over all 2^n basis states (a new tensor); for the
        complement-symmetric layout the stored half is expanded."""
        amps = self.amplitudes()
        if not self.symmetric:
            return amps
        torch = self.torch
        x = torch.arange(1 << self.n, dtype=torch.int64, device=self.device)
        top = (x >> (self.n - 1)) & 1
        y = torch.where(top == 1, x ^ ((1 << self.n) - 1), x)
        return amps[y ^ (y >> 1)]

    # ---- profiling
    def profile(self, enable: bool = True):
        _qs.qs_profile(self.handle, enable)

    def profile_read(self, kind: int):
        return _qs.qs_profile_read(self.handle, kind)

    def close(self):
        if self.handle is not None:
            _qs.qs_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mean_of_means(r_values, probs, n_shots: int, sigmas: float = 3.0):
    """Sec. II-D: the mean approximation ratio over n_shots bitstrings drawn
    from a distribution of r, summarised by its grand mean and spread.

    From the exact distribution (probs over r_values) the mean of n_shots
    independent draws has mean mu and standard deviation sigma / sqrt(n_shots);
    returns (mu, that spread, mu + sigmas * spread), the last being the
    threshold a measured mean must exceed.
    """
    r = np.asarray(r_values, dtype=np.float64)
    q = np.asarray(probs, dtype=np.float64)
    q = q / q.sum()
    mu = float((r * q).sum())
    sd = float(np.sqrt(max((((r - mu) ** 2) * q).sum(), 0.0)) / np.sqrt(n_shots))
    return mu, sd, mu + sigmas * sd


def _autograd():
    import torch

    class ExpectC(torch.autograd.Function):
        """<C>(gammas, betas) with the adjoint gradient of libqs.

        forward(gammas, betas, sim, convention, mode) runs the circuit and the
        reverse sweep once (mode "uncompute" or "store", see
        Simulator.adjoint); backward scales the stored gradient.
        """

        @staticmethod
        def forward(ctx, gammas, betas, sim, convention="paper", mode="uncompute"):
            g = gammas.detach().cpu().double().numpy()
            b = betas.detach().cpu().double().numpy()
            tzz, tx = to_gate_angles(g, b, convention)
            e, gzz, gx = sim.adjoint(tzz, tx, mode=mode)
            dg, db = gate_grad_to_schedule(gzz, gx, convention)
            ctx.save_for_backward(torch.as_tensor(dg, dtype=gammas.dtype),
                                  torch.as_tensor(db, dtype=betas.dtype))
            return torch.tensor(e, dtype=torch.float64)

        @staticmethod
        def backward(ctx, grad_out):
            dg, db = ctx.saved_tensors
            return grad_out.to(dg.dtype) * dg, grad_out.to(db.dtype) * db, None, None, None

    return ExpectC


_ExpectC = None


def expect_c(gammas, betas, sim: Simulator, convention: str = "paper", mode: str = "uncompute"):
    """Differentiable <C> as a function of per-layer (gamma_k, beta_k) CPU tensors;
    mode selects the adjoint's reverse sweep ("uncompute" or "store")."""
    global _ExpectC
    if _ExpectC is None:
        _ExpectC = _autograd()
    return _ExpectC.apply(gammas, betas, sim, convention, mode)


class Batch:
    """Many LR-QAOA circuits (own instance, depth and angles each) whose forward
    circuits and adjoint gradients run in one persistent kernel launch."""

    def __init__(self, instances, precision: str = "c64", stream=None):
        """instances: sequence of (w_tenths, p)."""
        import torch
        self.prec = PRECISIONS[precision]
        self.p = [int(p) for _, p in instances]
        self.n = [n_from_edges(len(w)) for w, _ in instances]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = _qs.qs_batch_create([(n, p, w) for n, (w, p) in zip(self.n, instances)], self.prec,
                                          self.stream)
        info = [_qs.qs_batch_info(self.handle, i) for i in range(len(self.n))]
        self.w_total = [x[0] for x in info]
        self.cmax = [x[1] for x in info]
        self.offsets = np.concatenate([[0], np.cumsum(self.p)])

    def forward_grad(self, theta_zz_list, theta_x_list):
        """Per-circuit gate angles -> (exp_c array, list of d_theta_zz, list of d_theta_x)."""
        tzz = np.concatenate([np.asarray(t, dtype=np.float64) for t in theta_zz_list])
        tx = np.concatenate([np.asarray(t, dtype=np.float64) for t in theta_x_list])
        e, gzz, gx = _qs.qs_batch_forward_grad(self.handle, tzz, tx, len(self.n))
        o = self.offsets
        return e, [gzz[o[i]:o[i + 1]] for i in range(len(self.n))], [gx[o[i]:o[i + 1]] for i in range(len(self.n))]

    def close(self):
        if self.handle is not None:
            _qs.qs_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trajectories:
    """Noisy LR-QAOA (Sec. II-C): a two-qubit depolarizing channel of rate eps
    after every RZZ gate, sampled as Pauli-insertion trajectories on the GPU
    (one workgroup per trajectory, n <= 12).  The mean of the per-trajectory
    <C> estimates <C> under the channel."""

    def __init__(self, w_tenths, precision: str = "c64", stream=None):
        import torch
        self.prec = PRECISIONS[precision]
        self.n = n_from_edges(len(w_tenths))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = _qs.qs_noise_create(self.n, self.prec, w_tenths, self.stream)
        self.w_total, self.cmax = _qs.qs_noise_info(self.handle)

    def run(self, theta_zz, theta_x, eps: float, seed: int, ntraj: int, traj0: int = 0, states: bool = False):
        """Trajectories traj0 .. traj0 + ntraj - 1 -> dict of device tensors:
        exp_c [ntraj] (units), norm [ntraj], nerr [ntraj] (non-identity Paulis)
        and, with states=True, the final states [ntraj, 2^n]."""
        import torch
        dev = torch.device("cuda")
        out = {"exp_c": torch.empty(ntraj, dtype=torch.float64, device=dev),
               "norm": torch.empty(ntraj, dtype=torch.float64, device=dev),
               "nerr": torch.empty(ntraj, dtype=torch.int32, device=dev)}
        if states:
            cdt = torch.complex64 if self.prec == _qs.QS_C64 else torch.complex128
            out["states"] = torch.empty((ntraj, 1 << self.n), dtype=cdt, device=dev)
        _qs.qs_noise_run(self.handle, theta_zz, theta_x, eps, seed, traj0, ntraj, out["exp_c"], out["norm"],
                         out["nerr"], out.get("states"))
        return out

    def ratio(self, theta_zz, theta_x, eps: float, seed: int, ntraj: int, traj0: int = 0):
        """(mean r, standard error of the mean) over the trajectories,
        r = <C> / C(x*) (eq. 5 with exact per-trajectory expectations)."""
        e = self.run(theta_zz, theta_x, eps, seed, ntraj, traj0)["exp_c"].double().cpu().numpy()
        r = e / (self.cmax / 10.0)
        return float(r.mean()), float(r.std(ddof=1) / np.sqrt(len(r))) if len(r) > 1 else 0.0

    def random_ratio(self) -> float:
        """Approximation ratio of the uniform random sampler: E[C] = W / 2."""
        return (self.w_total / 2.0) / self.cmax

    def close(self):
        if self.handle is not None:
            _qs.qs_noise_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

