"""PyTorch-facing API of libqva.

Tensors provide device memory and the current HIP stream; all arithmetic runs
in the library's HIP kernels.  Amplitudes are torch.complex128, qualities and
eigenvalues torch.float64, all on the same GPU.
"""

from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib

MIXERS = {"x": _lib.QVA_MIX_X, "circulant": _lib.QVA_MIX_CIRCULANT, "xy": _lib.QVA_MIX_XY}
LAMBDA_KINDS = {"array": _lib.QVA_LAMBDA_ARRAY, "ring": _lib.QVA_LAMBDA_RING,
                "complete": _lib.QVA_LAMBDA_COMPLETE}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None):
    return None if t is None else t.data_ptr()


def _need(t: torch.Tensor, dtype: torch.dtype, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _log2(N: int) -> int:
    n = int(N).bit_length() - 1
    if N < 1 or (1 << n) != N:
        raise ValueError(f"length {N} is not a power of two")
    return n


def _workspace(nbytes: int, device) -> torch.Tensor | None:
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- primitives
def init_uniform(psi: torch.Tensor) -> torch.Tensor:
    """psi <- N^(-1/2) (1, ..., 1), in place."""
    _need(psi, torch.complex128, "psi")
    _lib.check("qva_init_uniform", _lib.load().qva_init_uniform(_ptr(psi), psi.numel(), _stream()))
    return psi


def phase(psi: torch.Tensor, q: torch.Tensor, gamma: float) -> torch.Tensor:
    """psi <- exp(-i gamma q) psi, in place."""
    _need(psi, torch.complex128, "psi")
    _need(q, torch.float64, "q")
    if q.numel() != psi.numel():
        raise ValueError("q and psi differ in length")
    _lib.check("qva_phase", _lib.load().qva_phase(_ptr(psi), _ptr(q), psi.numel(), float(gamma),
                                                  _stream()))
    return psi


def mix_x(psi: torch.Tensor, t: float) -> torch.Tensor:
    """psi <- exp(-i t sum_i X_i) psi, in place."""
    _need(psi, torch.complex128, "psi")
    n = _log2(psi.numel())
    _lib.check("qva_mix_x", _lib.load().qva_mix_x(_ptr(psi), n, float(t), _stream()))
    return psi


def mix_circulant(psi: torch.Tensor, t: float, lam: torch.Tensor | None = None,
                  kind: str = "array") -> torch.Tensor:
    """psi <- F^-1 diag(exp(-i t lambda)) F psi, in place, for any N >= 2
    (kind "ring", "complete", or "array" with lam)."""
    _need(psi, torch.complex128, "psi")
    if kind == "array":
        _need(lam, torch.float64, "lam")
        if lam.numel() != psi.numel():
            raise ValueError("lam and psi differ in length")
    lib = _lib.load()
    ws = _workspace(lib.qva_mix_circulant_workspace_bytes(psi.numel()), psi.device)
    _lib.check("qva_mix_circulant",
               lib.qva_mix_circulant(_ptr(psi), _ptr(lam) if kind == "array" else None,
                                     LAMBDA_KINDS[kind], psi.numel(), float(t), _ptr(ws),
                                     0 if ws is None else ws.numel(), _stream()))
    return psi


def expectation(psi: torch.Tensor, q: torch.Tensor) -> tuple[torch.Tensor, torch.Tensor]:
    """(sum |psi|^2 q, sum |psi|^2) as 0-d float64 device tensors."""
    _need(psi, torch.complex128, "psi")
    _need(q, torch.float64, "q")
    if q.numel() != psi.numel():
        raise ValueError("q and psi differ in length")
    lib = _lib.load()
    out = torch.empty(2, dtype=torch.float64, device=psi.device)
    ws = _workspace(lib.qva_expectation_workspace_bytes(psi.numel()), psi.device)
    _lib.check("qva_expectation",
               lib.qva_expectation(_ptr(psi), _ptr(q), psi.numel(), out.data_ptr(),
                                   out.data_ptr() + 8, _ptr(ws), 0 if ws is None else ws.numel(),
                                   _stream()))
    return out[0], out[1]


# ------------------------------------------------------------- problem
class Problem:
    """A QVA instance: quality vector q (device float64) and the mixer.

    mixer "x": W = sum_i X_i on log2(len(q)) qubits.
    mixer "circulant": W circulant with eigenvalues lam (natural order) or
    lambda_kind "ring" / "complete".  A circulant may have any N >= 2 (the
    solution count of a constrained problem): closed-form passes for the
    complete graph; for the ring or an array, in-place mixed-radix passes
    when every prime factor of N is at most 31, else Bluestein's transform
    (both evolve and grad).  The hypercube mixer needs a power of two.

    terms (hypercube mixer only): the extended QAOA, one phase angle per term
    of a Z-string decomposition of the cost, given as (supports, coefs) with
    Sigma_e(j) = coefs[e] (-1)^popcount(j & supports[e]); gammas are then
    p x n_terms and q is only the observable.

    mixer "xy": the QAOAz parity mixer, the ordered product over `pairs`
    (a, b) of exp(-i t (X_a X_b + Y_a Y_b)), first pair first (see
    parity_ring_pairs), started from psi0 (a device complex128 state of the
    constrained subspace, e.g. a Dicke state).
    """

    def __init__(self, q: torch.Tensor, mixer: str = "x", lam: torch.Tensor | None = None,
                 lambda_kind: str = "array", terms=None, pairs=None, psi0: torch.Tensor | None = None):
        _need(q, torch.float64, "q")
        self.q = q
        N = q.numel()
        self._N = N
        if mixer == "circulant" and N >= 2 and (N & (N - 1)):
            self.n = int(N - 1).bit_length()  # log2 N rounded up
            n_states = N
        else:
            self.n = _log2(N)
            n_states = 0
        self.mixer = mixer
        self.lambda_kind = lambda_kind if mixer == "circulant" else "array"
        self.lam = lam
        if mixer == "circulant" and lambda_kind == "array":
            _need(lam, torch.float64, "lam")
            if lam.numel() != q.numel():
                raise ValueError("lam and q differ in length")
        self.terms = None
        self.n_terms = 0
        if terms is not None:
            supports, coefs = terms
            packed = np.zeros(len(supports), dtype=[("support", "<u8"), ("coef", "<f8")])
            packed["support"] = np.asarray(supports, dtype=np.uint64)
            packed["coef"] = np.asarray(coefs, dtype=np.float64)
            if len(packed) != len(coefs):
                raise ValueError("one coefficient per support")
            self.n_terms = len(packed)
            if self.n_terms:
                self.terms = torch.from_numpy(packed.view(np.uint8).copy()).to(q.device)
        self.pairs = None
        self.psi0 = None
        if mixer == "xy":
            self.pairs = np.ascontiguousarray(np.asarray(pairs if pairs is not None else [], dtype=np.int32)
                                              .reshape(-1, 2))
            _need(psi0, torch.complex128, "psi0")
            if psi0.numel() != N:
                raise ValueError("psi0 and q differ in length")
            self.psi0 = psi0
        self._c = _lib.QvaProblem(MIXERS[mixer], self.n, _ptr(q),
                                  _ptr(lam) if (mixer == "circulant" and lambda_kind == "array") else None,
                                  LAMBDA_KINDS[self.lambda_kind], n_states, _ptr(self.terms), self.n_terms,
                                  self.pairs.ctypes.data if self.pairs is not None and len(self.pairs) else None,
                                  0 if self.pairs is None else len(self.pairs))
        self.q_tiles = None
        self._q_version = q._version

    @property
    def N(self) -> int:
        return self._N

    @property
    def device(self):
        return self.q.device

    def cstruct(self):
        if self.q_tiles is not None and self.q._version != self._q_version:
            raise ValueError("q changed in place after tile_q(): call tile_q() again (or untile_q())")
        return ctypes.byref(self._c)

    def workspace_bytes(self, p: int, for_grad: bool = False) -> int:
        return int(_lib.load().qva_workspace_bytes(self.cstruct(), int(p), int(for_grad)))

    def tile_q(self) -> bool:
        """Write q in the hypercube passes' tile order (qva_q_tiles) and have
        every later call read it: a per-problem layout of the same values,
        one extra N-double block per qubit group.  Call again after changing q
        or the group split (an in-place change of q is caught through the
        tensor's version counter: calls then raise ValueError).  Returns False
        (and changes nothing) when this problem's passes do not read such a
        copy."""
        lib = _lib.load()
        self._c.q_tiles = None
        self._c.q_tiles_key = 0
        self.q_tiles = None
        self._q_version = self.q._version  # calls refuse the copy once q changes in place
        nbytes = int(lib.qva_q_tiles_bytes(self.cstruct()))
        if nbytes == 0:
            return False
        buf = torch.empty(nbytes // 8, dtype=torch.float64, device=self.q.device)
        key = ctypes.c_uint64(0)
        _lib.check("qva_q_tiles", lib.qva_q_tiles(self.cstruct(), buf.data_ptr(), nbytes, ctypes.byref(key),
                                                  _stream()))
        self.q_tiles = buf
        self._c.q_tiles = buf.data_ptr()
        self._c.q_tiles_key = key.value
        return True

    def untile_q(self) -> None:
        """Drop the tile-ordered copy of q (calls read q itself again)."""
        self._c.q_tiles = None
        self._c.q_tiles_key = 0
        self.q_tiles = None


def parity_ring_pairs(ring) -> list[tuple[int, int]]:
    """The factors of the QAOAz parity mixer (eqs. parity_terms, qaoaz_mixers)
    for a ring of qubits r_1..r_m, in the order they act: B_odd's pairs
    (r_a, r_a+1) for odd a, then B_even's for even a (r_m+1 is r_1), then B_last
    = (r_m, r_1) when m is odd."""
    r = [int(x) for x in ring]
    m = len(r)
    lib = _lib.load()
    ring_c = (ctypes.c_int * max(m, 1))(*r)
    cnt = lib.qva_parity_ring_pairs(ring_c, m, None, 0)
    _lib.check("qva_parity_ring_pairs", cnt if cnt < 0 else 0)
    out = (ctypes.c_int * max(2 * cnt, 1))()
    _lib.check("qva_parity_ring_pairs", min(lib.qva_parity_ring_pairs(ring_c, m, out, cnt), 0))
    return [(out[2 * i], out[2 * i + 1]) for i in range(cnt)]


def _angles(x, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        x = x.detach().to(device=device, dtype=torch.float64).contiguous()
        return x
    return torch.tensor(np.asarray(x, dtype=np.float64), dtype=torch.float64, device=device)


def _layer_angles(problem: Problem, gammas, ts, dev):
    """Flat device gammas (p, or p x n_terms with terms), ts and p."""
    g = _angles(gammas, dev).reshape(-1)
    t = _angles(ts, dev).reshape(-1)
    per = problem.n_terms if problem.n_terms > 0 else 1
    if g.numel() != t.numel() * per:
        raise ValueError("one gamma per layer (per term with terms) and one t per layer")
    return g, t, t.numel()


def evolve(problem: Problem, gammas, ts, psi: torch.Tensor | None = None, store: bool = True,
           workspace: torch.Tensor | None = None):
    """Run the p-layer evolution from the uniform state.

    Returns (f, norm, psi) with f, norm 0-d device tensors and psi the final
    state (a new tensor unless one is passed in).
    """
    dev = problem.device
    g, t, p = _layer_angles(problem, gammas, ts, dev)
    if psi is None:
        psi = torch.empty(problem.N, dtype=torch.complex128, device=dev)
    else:
        _need(psi, torch.complex128, "psi")
        if psi.numel() != problem.N:
            raise ValueError("psi has the wrong length")
    if problem.psi0 is not None:
        psi.copy_(problem.psi0)  # the XY mixer starts from the caller's state
    lib = _lib.load()
    need = problem.workspace_bytes(p)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    flags = 0 if store else _lib.QVA_EVOLVE_SKIP_FINAL_STATE
    _lib.check("qva_evolve",
               lib.qva_evolve(problem.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                              out.data_ptr(), out.data_ptr() + 8, flags, _ptr(workspace),
                              0 if workspace is None else workspace.numel(), _stream()))
    return out[0], out[1], psi


def evolve_noalloc(problem: Problem, gammas, ts, psi: torch.Tensor, out: torch.Tensor,
                   store: bool = True):
    """evolve() through qva_evolve_noalloc: the library's static per-device
    workspace instead of a caller one, so the call allocates nothing (for
    code under graph capture).  psi (N complex128) and out (2 float64:
    f, norm) are the caller's; angle tensors must already be float64 on the
    device.  Calls that overlap in time on one GPU race (one shared array)."""
    dev = problem.device
    _need(psi, torch.complex128, "psi")
    _need(out, torch.float64, "out")
    if psi.numel() != problem.N or out.numel() < 2:
        raise ValueError("psi must hold N amplitudes and out two doubles")
    g, t, p = _layer_angles(problem, gammas, ts, dev)
    if problem.psi0 is not None:
        psi.copy_(problem.psi0)
    flags = 0 if store else _lib.QVA_EVOLVE_SKIP_FINAL_STATE
    _lib.check("qva_evolve_noalloc",
               _lib.load().qva_evolve_noalloc(problem.cstruct(), g.data_ptr(), t.data_ptr(), p,
                                              psi.data_ptr(), out.data_ptr(), out.data_ptr() + 8, flags,
                                              _stream()))
    return out[0], out[1], psi


def grad(problem: Problem, gammas, ts, psi: torch.Tensor | None = None,
         chi: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """(f, df/dgamma, df/dt) by the adjoint method (device tensors); with
    terms, df/dgamma is p x n_terms."""
    dev = problem.device
    g, t, p = _layer_angles(problem, gammas, ts, dev)
    if psi is None:
        psi = torch.empty(problem.N, dtype=torch.complex128, device=dev)
    if chi is None:
        chi = torch.empty(problem.N, dtype=torch.complex128, device=dev)
    _need(psi, torch.complex128, "psi")
    _need(chi, torch.complex128, "chi")
    if psi.numel() != problem.N or chi.numel() != problem.N:
        raise ValueError("psi and chi must hold N amplitudes each")
    if problem.psi0 is not None:
        psi.copy_(problem.psi0)
    lib = _lib.load()
    need = problem.workspace_bytes(p, True)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    f = torch.empty((), dtype=torch.float64, device=dev)
    dg = torch.empty(g.numel(), dtype=torch.float64, device=dev)
    dt = torch.empty(p, dtype=torch.float64, device=dev)
    _lib.check("qva_grad",
               lib.qva_grad(problem.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                            chi.data_ptr(), f.data_ptr(), dg.data_ptr(), dt.data_ptr(),
                            _ptr(workspace), 0 if workspace is None else workspace.numel(),
                            _stream()))
    if problem.n_terms > 0:
        dg = dg.view(p, problem.n_terms)
    return f, dg, dt


class QVAExpectation(torch.autograd.Function):
    """f(gamma, t) = <psi_p|Q|psi_p> with the adjoint gradient as backward.

    forward runs the adjoint sweep at once (it yields f too) and saves the
    gradient; backward scales it by the incoming gradient.
    """

    @staticmethod
    def forward(ctx, gammas: torch.Tensor, ts: torch.Tensor, problem: Problem):
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            f, dg, dt = grad(problem, gammas, ts)
            ctx.save_for_backward(dg.reshape(gammas.shape), dt.reshape(ts.shape))
        else:
            f, _, _ = evolve(problem, gammas, ts, store=False)
            ctx.save_for_backward(None, None)
        return f.clone()

    @staticmethod
    def backward(ctx, grad_out):
        dg, dt = ctx.saved_tensors
        return (None if dg is None else grad_out * dg,
                None if dt is None else grad_out * dt, None)


def expectation_value(problem: Problem, gammas: torch.Tensor, ts: torch.Tensor) -> torch.Tensor:
    """Differentiable f(gamma, t) (float64 device tensors in, 0-d tensor out)."""
    return QVAExpectation.apply(gammas, ts, problem)


# ------------------------------------------------------------------ batched
_ALIGN = {"start": _lib.QVA_BATCH_ALIGN_START, "end": _lib.QVA_BATCH_ALIGN_END,
          "spread": _lib.QVA_BATCH_ALIGN_SPREAD}


class Batch:
    """Many independent QAOA instances (hypercube mixer): f and the adjoint
    gradient of all of them with one call, and a gradient-descent step.

    qs: list of device float64 quality vectors (lengths 2^n, 12 <= n <= 30);
    gammas, ts: lists of per-instance angle sequences (same length p_i).
    The angles live in two flat device tensors (`gammas`, `ts`) updated in
    place by `sgd`; results land in `f` (one per instance) and the flat
    `dgammas`, `dts` tensors (instance i at `offsets[i]:offsets[i] + p[i]`).
    `grad()` and `sgd()` only enqueue kernels on the current stream, so both
    can be captured into a torch.cuda.CUDAGraph and replayed.
    """

    def __init__(self, qs, gammas, ts, align: str = "spread", lanes: int = 1):
        if not (len(qs) == len(gammas) == len(ts)) or not qs:
            raise ValueError("one q, gammas and ts per instance")
        dev = qs[0].device
        self.count = len(qs)
        self.n = []
        self.p = [len(g) for g in gammas]
        self.offsets = []
        off = 0
        for g, t in zip(gammas, ts):
            if len(g) != len(t):
                raise ValueError("one gamma and one t per layer")
            self.offsets.append(off)
            off += len(g)
        self.gammas = torch.cat([_angles(g, dev) for g in gammas]).contiguous()
        self.ts = torch.cat([_angles(t, dev) for t in ts]).contiguous()
        self.dgammas = torch.zeros_like(self.gammas)
        self.dts = torch.zeros_like(self.ts)
        self.f = torch.zeros(self.count, dtype=torch.float64, device=dev)
        self.qs = []
        amp = 0
        amp_off = []
        for q in qs:
            _need(q, torch.float64, "q")
            self.qs.append(q)
            self.n.append(_log2(q.numel()))
            amp_off.append(amp)
            amp += q.numel()
        self.psi = torch.empty(amp, dtype=torch.complex128, device=dev)
        self.chi = torch.empty(amp, dtype=torch.complex128, device=dev)
        items = (_lib.QvaBatchItem * self.count)()
        for i in range(self.count):
            o, a = self.offsets[i], amp_off[i]
            items[i] = _lib.QvaBatchItem(
                self.n[i], self.p[i], self.qs[i].data_ptr(),
                self.gammas.data_ptr() + 8 * o, self.ts.data_ptr() + 8 * o,
                self.psi.data_ptr() + 16 * a, self.chi.data_ptr() + 16 * a,
                self.f.data_ptr() + 8 * i,
                self.dgammas.data_ptr() + 8 * o, self.dts.data_ptr() + 8 * o)
        lib = _lib.load()
        plan = ctypes.c_void_p()
        _lib.check("qva_batch_create_lanes",
                   lib.qva_batch_create_lanes(items, self.count, _ALIGN[align], int(lanes), ctypes.byref(plan)))
        self.lanes = int(lanes)
        self._plan = plan
        nbytes = lib.qva_batch_workspace_bytes(plan)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _lib.check("qva_batch_upload", lib.qva_batch_upload(plan, self.workspace.data_ptr(),
                                                            nbytes, _stream()))

    @property
    def rounds(self) -> int:
        return int(_lib.load().qva_batch_rounds(self._plan))

    @property
    def launches(self) -> int:
        return int(_lib.load().qva_batch_launches(self._plan))

    @property
    def tiles(self) -> int:
        return int(_lib.load().qva_batch_tiles(self._plan))

    def grad(self) -> None:
        """Enqueue f and the gradient of every instance."""
        lib = _lib.load()
        _lib.check("qva_batch_grad", lib.qva_batch_grad(self._plan, self.workspace.data_ptr(),
                                                        self.workspace.numel(), _stream()))

    def sgd(self, lr: float) -> None:
        """Enqueue gammas -= lr * dgammas, ts -= lr * dts."""
        lib = _lib.load()
        _lib.check("qva_batch_sgd", lib.qva_batch_sgd(self._plan, float(lr), self.workspace.data_ptr(),
                                                      self.workspace.numel(), _stream()))

    def instance(self, i: int):
        """(f, dgammas, dts) of instance i as device tensors (views)."""
        o, p = self.offsets[i], self.p[i]
        return self.f[i], self.dgammas[o:o + p], self.dts[o:o + p]

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            try:
                _lib.load().qva_batch_destroy(plan)
            except Exception:
                pass
            self._plan = None
