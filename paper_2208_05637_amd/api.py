"""Python binding of the nqs C ABI.

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch supplies device memory (tensors) and the stream
(``torch.cuda.current_stream()``).  Samples are uint64 bit strings; as torch
has few uint64 ops they travel as int64 tensors with the same bits.  A bit
string of n qubits is W = ceil(n / 64) words: samples are [B] for n <= 64 and
[B, 2] (word w = qubits 64w .. 64w+63) for 64 < n <= 128, and so are the
Pauli masks ([K] or [K, 2]).
"""
import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def words(n_qubits):
    """64-bit words per bit string of n qubits."""
    return (int(n_qubits) + 63) // 64


def _as_u64_tensor(x, device):
    if isinstance(x, torch.Tensor):
        if x.dtype not in (torch.int64, torch.uint64):
            raise TypeError("samples must be an int64/uint64 tensor of bit strings")
        return x.to(device).contiguous()
    arr = np.ascontiguousarray(np.asarray(x, dtype=np.uint64)).view(np.int64)
    return torch.from_numpy(arr.copy()).to(device)


def _strings(x, device, W):
    """(tensor, count) of bit strings of W words: [B] for W = 1, [B, W] else."""
    t = _as_u64_tensor(x, device)
    if W == 1:
        if t.dim() == 2 and t.shape[1] == 1:
            t = t.reshape(-1)
        if t.dim() != 1:
            raise ValueError("bit strings of at most 64 qubits are a 1-D array")
    elif t.dim() != 2 or t.shape[1] != W:
        raise ValueError(f"bit strings of more than 64 qubits are a [B, {W}] array of words")
    return t, t.shape[0]


def tune_db_load(path):
    """Add the tuner choices stored in path to this process's cache; returns the
    number of entries read."""
    n = C.c_int()
    L.check(L.load().nqs_tune_db_load(str(path).encode(), C.byref(n)), "nqs_tune_db_load")
    return n.value


def tune_db_save(path):
    """Write this process's tuner choices to path."""
    L.check(L.load().nqs_tune_db_save(str(path).encode()), "nqs_tune_db_save")


class Context:
    """A device + stream binding (no device memory is allocated)."""

    def __init__(self, device=0, stream=None):
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        L.check(self.lib.nqs_ctx_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h)),
                "nqs_ctx_create")
        self.handle = h

    def use_stream(self, stream):
        self.stream = stream
        L.check(self.lib.nqs_ctx_set_stream(self.handle, C.c_void_p(stream.cuda_stream)),
                "nqs_ctx_set_stream")

    def __del__(self):
        if getattr(self, "handle", None):
            self.lib.nqs_ctx_destroy(self.handle)
            self.handle = None


class Hamiltonian:
    """Pauli-string Hamiltonian canonicalised on the host (merge, drop, fold, sort, group)."""

    def __init__(self, n_qubits, x_mask, z_mask, coeff, coeff_imag=None, drop_tol=1e-10,
                 conserves_spin=True, tables=False):
        """tables: evaluate matrix elements from per-group structured tables (NQS_H_TABLES)."""
        self.lib = L.load()
        self.n = int(n_qubits)
        self.words = words(self.n)
        self._x = np.ascontiguousarray(np.asarray(x_mask, dtype=np.uint64))
        self._z = np.ascontiguousarray(np.asarray(z_mask, dtype=np.uint64))
        want = 1 if self.words == 1 else 2
        if self._x.ndim != want or self._z.shape != self._x.shape or (want == 2 and self._x.shape[1] != self.words):
            raise ValueError(f"masks of {self.n} qubits must be uint64 arrays of shape "
                             f"{'[K]' if want == 1 else f'[K, {self.words}]'}")
        self._c = np.ascontiguousarray(np.asarray(coeff, dtype=np.float64))
        self._ci = None if coeff_imag is None else np.ascontiguousarray(np.asarray(coeff_imag, dtype=np.float64))
        t = L.PauliTerms(self.n, self._x.shape[0], self._x.ctypes.data, self._z.ctypes.data,
                         self._c.ctypes.data, None if self._ci is None else self._ci.ctypes.data,
                         float(drop_tol), (L.NQS_H_CONSERVES_SPIN_SECTORS if conserves_spin else 0)
                         | (L.NQS_H_TABLES if tables else 0))
        h = C.c_void_p()
        L.check(self.lib.nqs_ham_create(C.byref(t), C.byref(h)), "nqs_ham_create")
        self.handle = h
        K, G, nb = C.c_int64(), C.c_int64(), C.c_size_t()
        im, nq = C.c_int(), C.c_int()
        L.check(self.lib.nqs_ham_info(h, C.byref(K), C.byref(G), C.byref(nb), C.byref(im), C.byref(nq)),
                "nqs_ham_info")
        self.K, self.G, self.bytes, self.has_imag = K.value, G.value, nb.value, bool(im.value)
        self.storage = None

    @classmethod
    def from_terms(cls, terms, **kw):
        return cls(terms.n_qubits, terms.x_mask, terms.z_mask, terms.coeff, **kw)

    def upload(self, ctx):
        self.storage = torch.empty(self.bytes + 256, dtype=torch.uint8, device=ctx.device)
        base = self.storage.data_ptr()
        aligned = (base + 255) & ~255
        L.check(self.lib.nqs_ham_upload(self.handle, ctx.handle, C.c_void_p(aligned), self.bytes),
                "nqs_ham_upload")
        return self

    def export(self):
        shape = (lambda m: (m,)) if self.words == 1 else (lambda m: (m, self.words))
        gx = np.zeros(shape(self.G), dtype=np.uint64)
        goff = np.zeros(self.G + 1, dtype=np.int64)
        tz = np.zeros(shape(self.K), dtype=np.uint64)
        tre = np.zeros(self.K, dtype=np.float64)
        tim = np.zeros(self.K, dtype=np.float64)
        L.check(self.lib.nqs_ham_export(self.handle, gx.ctypes.data, goff.ctypes.data, tz.ctypes.data,
                                        tre.ctypes.data, tim.ctypes.data), "nqs_ham_export")
        return dict(gx=gx, goff=goff, tz=tz, tre=tre, tim=tim)

    def export_tables(self):
        """Host copy of the structured tables (empty arrays without NQS_H_TABLES)."""
        S, E = C.c_int64(), C.c_int64()
        L.check(self.lib.nqs_ham_table_info(self.handle, C.byref(S), C.byref(E)), "nqs_ham_table_info")
        S, E = S.value, E.value
        # soff and fpos are sized by the groups: a table Hamiltonian without terms still has soff[0]
        soff = np.zeros(self.G + 1, dtype=np.int64)
        su = np.zeros((S, self.words), dtype=np.uint64)
        stab = np.zeros(S, dtype=np.int64)
        tre = np.zeros(E, dtype=np.float64)
        tim = np.zeros(E, dtype=np.float64)
        fpos = np.zeros((self.G, 4), dtype=np.int8)
        L.check(self.lib.nqs_ham_export_tables(self.handle, soff.ctypes.data, su.ctypes.data, stab.ctypes.data,
                                               tre.ctypes.data, tim.ctypes.data, fpos.ctypes.data),
                "nqs_ham_export_tables")
        return dict(soff=soff, su=su, stab=stab, tre=tre, tim=tim, fpos=fpos)

    def __del__(self):
        if getattr(self, "handle", None):
            self.lib.nqs_ham_destroy(self.handle)
            self.handle = None


def net_desc(n_qubits, n_layers, width, n_up=-1, n_dn=-1, precision="fp32", order=None, phase_mode=0):
    """phase_mode: 0 (or "shared") phase head on the masked trunk; 1 (or
    "separate") the separate phase sub-model."""
    order_arr = None
    if order is not None:
        order_arr = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    pm = {"shared": 0, "separate": 1}.get(phase_mode, phase_mode)
    d = L.NetDesc(int(n_qubits), int(n_layers), int(width),
                  None if order_arr is None else order_arr.ctypes.data, int(n_up), int(n_dn),
                  L.PRECISIONS[precision] if isinstance(precision, str) else int(precision), int(pm))
    return d, order_arr


def param_count(n_qubits, n_layers, width, precision="fp32", phase_mode=0):
    lib = L.load()
    d, keep = net_desc(n_qubits, n_layers, width, precision=precision, phase_mode=phase_mode)
    out = C.c_int64()
    L.check(lib.nqs_net_param_count(C.byref(d), C.byref(out)), "nqs_net_param_count")
    return out.value


class Plan:
    """Kernel variants, chunking and workspace layout for one (H, network) pair."""

    def __init__(self, ctx, ham, n_layers, width, n_up=-1, n_dn=-1, precision="fp32",
                 max_batch=1024, dedup=False, chunk_samples=0, order=None, phase_mode=0):
        """dedup: True, False or "auto" (the autotuner decides); phase_mode as in net_desc."""
        self.lib = L.load()
        self.ctx, self.ham = ctx, ham
        self.words = ham.words
        self.precision = precision
        d, self._order = net_desc(ham.n, n_layers, width, n_up, n_dn, precision, order, phase_mode)
        if dedup == "auto":
            flags = L.NQS_PLAN_DEDUP_AUTO
        else:
            flags = L.NQS_PLAN_DEDUP_ON if dedup else L.NQS_PLAN_DEDUP_OFF
        h = C.c_void_p()
        L.check(self.lib.nqs_plan_create(ctx.handle, ham.handle, C.byref(d), int(max_batch), flags,
                                         int(chunk_samples), C.byref(h)), "nqs_plan_create")
        self.handle = h
        self.max_batch = int(max_batch)
        self._ws = None
        self._refresh()

    def _refresh(self):
        e, cs, dd, npar = C.c_int64(), C.c_int64(), C.c_int(), C.c_int64()
        L.check(self.lib.nqs_plan_info(self.handle, C.byref(e), C.byref(cs), C.byref(dd), C.byref(npar)),
                "nqs_plan_info")
        self.entries_per_sample, self.chunk_samples = e.value, cs.value
        self.dedup, self.n_params = bool(dd.value), npar.value

    def configure(self, waves_per_block=0, dedup=None, chunk_samples=0, resident=None, rows_per_block=0):
        """Set the forward's workgroup shape (waves per workgroup, rows per tile),
        dedup, chunk and the forward's grid (resident workgroups looping over
        tiles) by hand; 0 / None keep the current value."""
        d = -1 if dedup is None else (1 if dedup else 0)
        r = -1 if resident is None else (1 if resident else 0)
        L.check(self.lib.nqs_plan_configure(self.handle, int(waves_per_block), int(rows_per_block), d,
                                            int(chunk_samples), r), "nqs_plan_configure")
        self._refresh()

    def kernel_info(self):
        """(waves per workgroup, configurations per workgroup, tuned, resident grid) of the forward."""
        w, r, t, g = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        L.check(self.lib.nqs_plan_kernel_info(self.handle, C.byref(w), C.byref(r), C.byref(t), C.byref(g)),
                "nqs_plan_kernel_info")
        return dict(waves_per_block=w.value, rows_per_block=r.value, tuned=bool(t.value), resident=bool(g.value))

    def autotune(self, params, samples, force=False, cache_only=False):
        """Time the candidate kernel variants / dedup / chunk sizes on a prefix of
        the samples and keep the fastest; returns the timings.  cache_only:
        apply a cached (or database) choice if there is one, never time."""
        params = _params(self, params)
        x, B = _strings(samples, self.ctx.device, self.words)
        rep = L.TuneReport()
        ws, nb = self.workspace()
        flags = (L.NQS_TUNE_FORCE if force else 0) | (L.NQS_TUNE_CACHE_ONLY if cache_only else 0)
        L.check(self.lib.nqs_plan_autotune(self.handle, _ptr(params), _ptr(x), B, ws, nb, flags, C.byref(rep)),
                "nqs_plan_autotune")
        self._refresh()
        cands = [dict(waves_per_block=c.waves_per_block, rows_per_block=c.rows_per_block, dedup=bool(c.dedup),
                      chunk_samples=c.chunk_samples, resident=bool(c.resident), ms=c.ms)
                 for c in rep.cand[:rep.n_candidates]]
        return dict(candidates=cands, chosen=rep.chosen, from_cache=bool(rep.from_cache),
                    probe_samples=rep.probe_samples)

    def workspace_size(self, B):
        out = C.c_size_t()
        L.check(self.lib.nqs_plan_workspace_size(self.handle, int(B), C.byref(out)),
                "nqs_plan_workspace_size")
        return out.value

    def workspace(self, B=None):
        """A cached device workspace large enough for batch B (default: max_batch)."""
        need = self.workspace_size(self.max_batch if B is None else B)
        if self._ws is None or self._ws[1] < need:
            raw = torch.empty(need + 256, dtype=torch.uint8, device=self.ctx.device)
            aligned = (raw.data_ptr() + 255) & ~255
            self._ws = (raw, need, aligned)
        return C.c_void_p(self._ws[2]), self._ws[1]

    def profile(self, enable=True):
        L.check(self.lib.nqs_plan_profile(self.handle, 1 if enable else 0), "nqs_plan_profile")

    def profile_read(self):
        """Totals since the last read: calls, call/eloc/forward ms, forward rows and flops."""
        out = L.Profile()
        ws, _ = self.workspace()
        L.check(self.lib.nqs_plan_profile_read(self.handle, ws, C.byref(out)), "nqs_plan_profile_read")
        return {f: getattr(out, f) for f, _ in L.Profile._fields_}

    def __del__(self):
        if getattr(self, "handle", None):
            self.lib.nqs_plan_destroy(self.handle)
            self.handle = None


def _dev_tensor(t, name, dtypes, numel, device):
    """Reject a tensor the kernels would read or write out of bounds."""
    if not isinstance(dtypes, tuple):
        dtypes = (dtypes,)
    if (not isinstance(t, torch.Tensor) or t.dtype not in dtypes or t.device != torch.device(device)
            or not t.is_contiguous() or t.numel() != numel):
        raise ValueError(f"{name} must be a contiguous {'/'.join(map(str, dtypes))} tensor of {numel} "
                         f"elements on {device}")
    return t


def _params(plan, params):
    if params.dtype != torch.float32 or not params.is_cuda or params.numel() != plan.n_params:
        raise ValueError(f"params must be a float32 CUDA tensor of {plan.n_params} entries")
    return params.contiguous()


def log_psi(plan, params, x):
    params = _params(plan, params)
    x, B = _strings(x, plan.ctx.device, plan.words)
    out = torch.empty((B, 2), dtype=torch.float64, device=plan.ctx.device)
    ws, nb = plan.workspace()
    L.check(plan.lib.nqs_log_psi(plan.handle, _ptr(params), _ptr(x), B, _ptr(out), ws, nb),
            "nqs_log_psi")
    return out


def local_energy(plan, params, samples):
    params = _params(plan, params)
    x, B = _strings(samples, plan.ctx.device, plan.words)
    out = torch.empty((B, 2), dtype=torch.float64, device=plan.ctx.device)
    ws, nb = plan.workspace()
    L.check(plan.lib.nqs_local_energy(plan.handle, _ptr(params), _ptr(x), B, _ptr(out), ws, nb),
            "nqs_local_energy")
    return out


def energy_grad(plan, params, samples, weights=None, eloc=None, energy=None, grad=None):
    """(energy[3] = (E, Im mean, W), grad f64 [n_params], eloc [B,2]) on the device."""
    params = _params(plan, params)
    dev = plan.ctx.device
    x, B = _strings(samples, dev, plan.words)
    w = None
    if weights is not None:
        w = _dev_tensor(torch.as_tensor(weights, dtype=torch.float64).to(dev).contiguous(), "weights",
                        torch.float64, B, dev)
    eloc = torch.empty((B, 2), dtype=torch.float64, device=dev) if eloc is None else eloc
    energy = torch.empty(3, dtype=torch.float64, device=dev) if energy is None else energy
    grad = torch.empty(plan.n_params, dtype=torch.float64, device=dev) if grad is None else grad
    _dev_tensor(eloc, "eloc", torch.float64, 2 * B, dev)
    _dev_tensor(energy, "energy", torch.float64, 3, dev)
    _dev_tensor(grad, "grad", torch.float64, plan.n_params, dev)
    ws, nb = plan.workspace()
    L.check(plan.lib.nqs_energy_grad(plan.handle, _ptr(params), _ptr(x), _ptr(w), B, _ptr(eloc),
                                     _ptr(energy), _ptr(grad), ws, nb), "nqs_energy_grad")
    return energy, grad, eloc


def energy_grad_noalloc(plan, params, samples, weights=None, eloc=None, energy=None, grad=None, flags=None):
    """energy_grad on the library's own static device workspace (no workspace
    tensor): for callers that cannot allocate, e.g. under graph capture with
    every output passed in.  Returns (energy, grad, eloc, flags), flags a
    uint32 device tensor (viewed as int32) holding the call's error word."""
    params = _params(plan, params)
    dev = plan.ctx.device
    x, B = _strings(samples, dev, plan.words)
    w = None
    if weights is not None:
        w = _dev_tensor(torch.as_tensor(weights, dtype=torch.float64).to(dev).contiguous(), "weights",
                        torch.float64, B, dev)
    eloc = torch.empty((B, 2), dtype=torch.float64, device=dev) if eloc is None else eloc
    energy = torch.empty(3, dtype=torch.float64, device=dev) if energy is None else energy
    grad = torch.empty(plan.n_params, dtype=torch.float64, device=dev) if grad is None else grad
    flags = torch.empty(1, dtype=torch.int32, device=dev) if flags is None else flags
    _dev_tensor(eloc, "eloc", torch.float64, 2 * B, dev)
    _dev_tensor(energy, "energy", torch.float64, 3, dev)
    _dev_tensor(grad, "grad", torch.float64, plan.n_params, dev)
    _dev_tensor(flags, "flags", torch.int32, 1, dev)
    L.check(plan.lib.nqs_energy_grad_noalloc(plan.handle, _ptr(params), _ptr(x), _ptr(w), B, _ptr(eloc),
                                             _ptr(energy), _ptr(grad), _ptr(flags)), "nqs_energy_grad_noalloc")
    return energy, grad, eloc, flags


def _instances(items):
    arr = (L.Instance * len(items))()
    for i, it in enumerate(items):
        plan, dev = it["plan"], it["plan"].ctx.device
        B = it["samples"].shape[0]
        _dev_tensor(it["params"], "params", torch.float32, plan.n_params, dev)
        _dev_tensor(it["samples"], "samples", (torch.int64, torch.uint64), B * plan.words, dev)
        if it.get("weights") is not None:
            _dev_tensor(it["weights"], "weights", torch.float64, B, dev)
        if it.get("eloc") is not None:
            _dev_tensor(it["eloc"], "eloc", torch.float64, 2 * B, dev)
        _dev_tensor(it["energy"], "energy", torch.float64, 3, dev)
        _dev_tensor(it["grad"], "grad", torch.float64, plan.n_params, dev)
        arr[i] = L.Instance(it["plan"].handle.value, it["params"].data_ptr(), it["samples"].data_ptr(),
                            it["weights"].data_ptr() if it.get("weights") is not None else None,
                            B,
                            it["eloc"].data_ptr() if it.get("eloc") is not None else None,
                            it["energy"].data_ptr(), it["grad"].data_ptr())
    return arr


def multi_workspace(items):
    """A device workspace for energy_grad_multi over items: (raw tensor, pointer, bytes)."""
    lib = L.load()
    need = C.c_size_t()
    L.check(lib.nqs_multi_workspace_size(len(items), _instances(items), C.byref(need)), "nqs_multi_workspace_size")
    raw = torch.empty(need.value + 256, dtype=torch.uint8, device=items[0]["plan"].ctx.device)
    return raw, C.c_void_p((raw.data_ptr() + 255) & ~255), need.value


def energy_grad_multi(items, workspace=None):
    """items: list of dicts with plan, params, samples, weights, eloc, energy, grad tensors.
    workspace: as returned by multi_workspace (allocated here when None)."""
    if workspace is None:
        workspace = multi_workspace(items)
    _, ws, nb = workspace
    lib = L.load()
    L.check(lib.nqs_energy_grad_multi(len(items), _instances(items), ws, nb), "nqs_energy_grad_multi")


def multi_device_status(items, workspace):
    """Device error words (or-ed) of a multi-instance call's instances, read and cleared."""
    _, ws, _ = workspace
    lib = L.load()
    flags = C.c_uint32()
    st = lib.nqs_multi_device_status(len(items), _instances(items), ws, C.byref(flags))
    if st not in (L.NQS_OK, 6):
        L.check(st, "nqs_multi_device_status")
    return flags.value


def sample(plan, params, n_draws, seed, max_unique):
    """Unique-sample autoregressive sampling (Sec. 4): (x int64 [U] or [U, W], weights f64 [U])."""
    params = _params(plan, params)
    dev = plan.ctx.device
    need = C.c_size_t()
    L.check(plan.lib.nqs_sample_workspace_size(plan.handle, int(max_unique), C.byref(need)),
            "nqs_sample_workspace_size")
    raw = torch.empty(need.value + 256, dtype=torch.uint8, device=dev)
    ws = C.c_void_p((raw.data_ptr() + 255) & ~255)
    x = torch.empty(int(max_unique) if plan.words == 1 else (int(max_unique), plan.words), dtype=torch.int64,
                    device=dev)
    w = torch.empty(int(max_unique), dtype=torch.float64, device=dev)
    nu = torch.zeros(1, dtype=torch.int64, device=dev)
    L.check(plan.lib.nqs_sample(plan.handle, _ptr(params), int(n_draws), int(seed) & (2**64 - 1),
                                int(max_unique), _ptr(x), _ptr(w), _ptr(nu), ws, need.value), "nqs_sample")
    U = int(nu.item())
    return x[:U], w[:U]


def connected(plan, samples, capacity=None):
    dev = plan.ctx.device
    x, B = _strings(samples, dev, plan.words)
    cap = int(capacity if capacity is not None else max(1, B * plan.entries_per_sample))
    out = dict(
        diag=torch.empty((B, 2), dtype=torch.float64, device=dev),
        sample=torch.empty(cap, dtype=torch.int32, device=dev),
        x=torch.empty(cap if plan.words == 1 else (cap, plan.words), dtype=torch.int64, device=dev),
        h=torch.empty((cap, 2), dtype=torch.float64, device=dev),
        n_entries=torch.zeros(1, dtype=torch.int64, device=dev),
    )
    if plan.dedup:
        out.update(unique=torch.empty(cap if plan.words == 1 else (cap, plan.words), dtype=torch.int64, device=dev),
                   entry_unique=torch.empty(cap, dtype=torch.int32, device=dev),
                   n_unique=torch.zeros(1, dtype=torch.int64, device=dev))
    ws, nb = plan.workspace()
    L.check(plan.lib.nqs_connected(plan.handle, _ptr(x), B, cap, _ptr(out["diag"]), _ptr(out["sample"]),
                                   _ptr(out["x"]), _ptr(out["h"]), _ptr(out["n_entries"]),
                                   _ptr(out.get("unique")), _ptr(out.get("entry_unique")),
                                   _ptr(out.get("n_unique")), ws, nb), "nqs_connected")
    return out


def reduce_table(plan, logpsi_samples, logpsi_entries, diag, entry_sample, entry_h, n_entries):
    dev = plan.ctx.device
    B = logpsi_samples.shape[0]
    eloc = torch.empty((B, 2), dtype=torch.float64, device=dev)
    ws, nb = plan.workspace()
    L.check(plan.lib.nqs_reduce_table(plan.handle, B, _ptr(logpsi_samples.contiguous()),
                                      _ptr(logpsi_entries.contiguous()), _ptr(diag.contiguous()),
                                      _ptr(entry_sample.contiguous()), _ptr(entry_h.contiguous()),
                                      int(n_entries), _ptr(eloc), ws, nb), "nqs_reduce_table")
    return eloc


def device_status(plan):
    ws, _ = plan.workspace()
    flags = C.c_uint32()
    st = plan.lib.nqs_device_status(plan.ctx.handle, ws, C.byref(flags))
    if st not in (L.NQS_OK, 6):
        L.check(st, "nqs_device_status")
    return flags.value


class Adam:
    """Adam on the flat FP32 parameter tensor (Sec. 6), one nqs_adam_step per
    call; the FP64 moments are torch tensors owned by this object."""

    def __init__(self, ctx, params, lr=1e-3, betas=(0.9, 0.99), eps=1e-8):
        if params.dtype != torch.float32 or not params.is_contiguous():
            raise TypeError("params must be a contiguous float32 tensor")
        self.ctx, self.params = ctx, params
        self.lr, self.betas, self.eps = float(lr), (float(betas[0]), float(betas[1])), float(eps)
        self.m = torch.zeros(params.numel(), dtype=torch.float64, device=params.device)
        self.v = torch.zeros_like(self.m)
        self.t = 0

    def step(self, grad):
        if grad.dtype != torch.float64 or grad.numel() != self.params.numel() or not grad.is_contiguous():
            raise TypeError("grad must be a contiguous float64 tensor of the parameters' size")
        self.t += 1
        L.check(self.ctx.lib.nqs_adam_step(self.ctx.handle, self.params.numel(), _ptr(self.params), _ptr(grad),
                                           _ptr(self.m), _ptr(self.v), self.t, self.lr, self.betas[0],
                                           self.betas[1], self.eps), "nqs_adam_step")


class EnergyFn(torch.autograd.Function):
    """(E, eloc) = EnergyFn.apply(params, samples, weights, plan).

    backward returns dL/dE * g with g the VMC gradient of E = <H> (Eq. grad
    with baseline E, times 2); the local energies are treated as constants,
    so this is the estimator, not autodiff of the returned estimate.
    """

    @staticmethod
    def forward(ctx, params, samples, weights, plan):
        energy, grad, eloc = energy_grad(plan, params, samples, weights)
        ctx.save_for_backward(grad)
        return energy[0].clone(), eloc

    @staticmethod
    def backward(ctx, g_energy, g_eloc):
        (grad,) = ctx.saved_tensors
        return (g_energy * grad).to(torch.float32), None, None, None
