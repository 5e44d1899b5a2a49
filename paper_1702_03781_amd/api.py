"""Python binding of libharp: argument marshalling only.

Every numerical step runs in the HIP library; PyTorch provides device memory
and the current stream.  Function names follow the C ABI (include/harp.h).

Matrices are returned as column-major views: a batch of n x m matrices is a
tensor ``M`` of shape (batch, n, m) with ``M.stride() == (s, 1, ld)``, which
is what the library reads and writes (ld = leading dimension).
"""
from __future__ import annotations

import ctypes
import math
import struct
import time
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import HarpElement, HarpError, HarpRefine, HarpRefineReport, HarpTuningEntry, check, lib

C64, C128 = 0, 1
# status codes of include/harp.h raised by the binding after reading the
# device-side outcome flags
HARP_E_ARG, HARP_E_DOMAIN, HARP_E_SINGULAR = -1, -2, -3
_DT = {"c64": C64, "c128": C128, torch.complex64: C64, torch.complex128: C128}
_TORCH_DT = {C64: torch.complex64, C128: torch.complex128}


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def colmajor(batch: int, rows: int, cols: int, dtype, device) -> torch.Tensor:
    """Allocate a batch of column-major matrices (ld = rows)."""
    return torch.empty((batch, cols, rows), dtype=dtype, device=device).transpose(1, 2)


def _cm(M: torch.Tensor, name: str):
    """(ptr, ld, stride) of a batched column-major tensor (batch, rows, cols)."""
    if M.dim() == 2:
        M = M.unsqueeze(0)
    if M.dim() != 3 or not M.is_cuda:
        raise ValueError(f"{name}: expected a CUDA tensor (batch, rows, cols)")
    b, r, c = M.shape
    if M.stride(1) != 1 and r > 1:
        raise ValueError(f"{name}: not column-major (stride {M.stride()})")
    ld = M.stride(2) if c > 1 else r
    if ld < r:
        raise ValueError(f"{name}: leading dimension {ld} < rows {r}")
    stride = M.stride(0) if b > 1 else ld * c
    return _ptr(M), ld, stride


def check_flags(fill_info=None, factor_info=None, where: str = "") -> None:
    """Raise the library's numerical outcomes as errors (reads the device
    flags, so it waits for the work that writes them).  fill_info: pairs
    closer than the model's inner radius r_min (HARP_E_DOMAIN), or -1 / -2 for
    a model or descriptor that does not match (HARP_E_ARG); factor_info: the
    1-based index of an exact zero pivot (HARP_E_SINGULAR)."""
    def host(v):
        return v.detach().cpu().numpy().ravel() if hasattr(v, "detach") else np.asarray(v).ravel()

    if fill_info is not None:
        fi = host(fill_info)
        if (fi < 0).any():
            raise HarpError(HARP_E_ARG, f"{where}: model or system descriptor mismatch "
                                        f"(entries {np.flatnonzero(fi < 0).tolist()})")
        if (fi > 0).any():
            raise HarpError(HARP_E_DOMAIN, f"{where}: {int(fi.sum())} antenna pair(s) closer than the "
                                           f"model's r_min (matrices {np.flatnonzero(fi > 0).tolist()})")
    if factor_info is not None:
        ii = host(factor_info)
        if (ii > 0).any():
            b = int(np.flatnonzero(ii > 0)[0])
            raise HarpError(HARP_E_SINGULAR, f"{where}: exact zero pivot at column {int(ii[b]) - 1} "
                                             f"of matrix {b}")


# --------------------------------------------------------------------------
# models
# --------------------------------------------------------------------------

_HDR = struct.Struct("<II6i5d6q")


@dataclass
class Model:
    """One HARP model (one element type at one frequency) in device memory."""
    blob: torch.Tensor      # uint8, device
    n_mbf: int
    n_samp: int
    P: int
    Q: int
    freq: float
    r_min: float
    # reciprocity of the table (C^{ST}_p = (-1)^p C^{TS}_p, Z_self = Z_self^T),
    # which makes the filled matrix complex-symmetric; harp_fit guarantees it
    # (even angular grid), pack_model measures it
    reciprocal: bool = True

    @property
    def nbytes(self) -> int:
        return int(self.blob.numel())


def model_bytes(n_mbf: int, n_samp: int, P: int, Q: int) -> int:
    return int(lib().harp_model_bytes(n_mbf, n_samp, P, Q))


def harp_fit(samples: torch.Tensor, wire_radius: float, freq: float, P: int, Q: int,
             r_min: float, n_alpha: int | None = None, n_t: int | None = None) -> Model:
    """Build the model of an element (device samples [n_mbf, n_samp, 8] f64)."""
    if samples.dtype != torch.float64 or not samples.is_cuda or samples.dim() != 3:
        raise ValueError("samples: CUDA float64 tensor [n_mbf, n_samp, 8]")
    samples = samples.contiguous()
    n_mbf, n_samp = samples.shape[0], samples.shape[1]
    n_alpha = 4 * (P + 1) if n_alpha is None else n_alpha
    n_t = 2 * (Q + 1) if n_t is None else n_t
    nb = model_bytes(n_mbf, n_samp, P, Q)
    blob = torch.zeros(nb, dtype=torch.uint8, device=samples.device)
    ws_b = ctypes.c_size_t()
    check(lib().harp_fit_ws(n_mbf, n_samp, P, Q, n_alpha, n_t, ctypes.byref(ws_b)), "harp_fit_ws")
    ws = torch.empty(max(1, ws_b.value), dtype=torch.uint8, device=samples.device)
    el = HarpElement(n_mbf, n_samp, _ptr(samples), float(wire_radius))
    check(lib().harp_fit(ctypes.byref(el), float(freq), P, Q, float(r_min), n_alpha, n_t,
                         _ptr(blob), nb, _ptr(ws), ws_b.value, _stream(samples.device)),
          "harp_fit")
    blob._keep = (samples, ws)  # keep inputs alive until the stream has consumed them
    return Model(blob, n_mbf, n_samp, P, Q, float(freq), float(r_min))


def pack_model(C: np.ndarray, Z_self: np.ndarray, w: np.ndarray, samples: np.ndarray,
               freq: float, k: float, omega_mu: float, r_min: float, wire_radius: float,
               device="cuda") -> Model:
    """Write a model blob (layout of include/harp.h) from host arrays, e.g. a
    table produced by another fitter or loaded from disk."""
    n_mbf, _, np2, q1 = C.shape
    P, Q = (np2 - 1) // 2, q1 - 1
    n_samp = samples.shape[1]
    total = model_bytes(n_mbf, n_samp, P, Q)

    def a256(b):
        return (b + 255) & ~255

    ncoef = n_mbf * n_mbf * np2 * q1
    off_coef = 256
    off_coef32 = off_coef + a256(ncoef * 16)
    off_self = off_coef32 + a256(ncoef * 8)
    off_port = off_self + a256(n_mbf * n_mbf * 16)
    off_samples = off_port + a256(n_mbf * 16)
    buf = np.zeros(total, dtype=np.uint8)
    hdr = _HDR.pack(0x50524148, 1, n_mbf, n_samp, P, Q, 0, 0, freq, k, omega_mu, r_min,
                    wire_radius, off_coef, off_coef32, off_self, off_port, off_samples, total)
    buf[:len(hdr)] = np.frombuffer(hdr, dtype=np.uint8)

    def put(off, arr):
        b = np.ascontiguousarray(arr).view(np.uint8).ravel()
        buf[off:off + b.size] = b

    put(off_coef, C.astype(np.complex128))
    put(off_coef32, C.astype(np.complex64))
    put(off_self, Z_self.astype(np.complex128))
    put(off_port, w.astype(np.complex128))
    put(off_samples, samples.astype(np.float64))
    blob = torch.from_numpy(buf).to(device)
    return Model(blob, n_mbf, n_samp, P, Q, float(freq), float(r_min), _table_reciprocal(C, Z_self))


def _table_reciprocal(C: np.ndarray, Z_self: np.ndarray) -> bool:
    """C^{ST}_pq = (-1)^p C^{TS}_pq and Z_self = Z_self^T (to rounding of a fit)."""
    P = (C.shape[2] - 1) // 2
    sign = (-1.0) ** np.arange(-P, P + 1)
    scale = max(float(np.abs(C).max()), 1e-300)
    return bool(np.abs(np.swapaxes(C, 0, 1) - sign[None, None, :, None] * C).max() <= 1e-8 * scale and
                np.abs(Z_self - Z_self.T).max() <= 1e-12 * max(float(np.abs(Z_self).max()), 1e-300))


# --------------------------------------------------------------------------
# persisted models (a model is built once per element and frequency and
# reused for every layout, Section III-C)
# --------------------------------------------------------------------------

_FILE_MAGIC = b"HARPMODL"
_FILE_VERSION = 1
_FILE_HDR = struct.Struct("<8sII32sQ")   # magic, file version, blob version, element hash, blob bytes


def element_hash(samples: np.ndarray, wire_radius: float) -> bytes:
    """SHA-256 of an element description: the [n_mbf][n_samp][8] float64
    sample records (little-endian) and the wire radius."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(samples, dtype="<f8").tobytes())
    h.update(struct.pack("<d", float(wire_radius)))
    return h.digest()


def _blob_element_hash(raw: np.ndarray) -> bytes:
    vals = _HDR.unpack(bytes(raw[:_HDR.size]))
    nm, ns, wire, off_s = vals[2], vals[3], vals[12], vals[17]
    samples = raw[off_s:off_s + nm * ns * 8 * 8].view("<f8").reshape(nm, ns, 8)
    return element_hash(samples, wire)


def save_model(model: Model, path: str) -> None:
    """Write a model blob to `path`: a 56-byte file header (magic "HARPMODL",
    file version, blob version, SHA-256 of the element the blob was built
    from, blob size) followed by the blob bytes exactly as the library reads
    them."""
    raw = model.blob.detach().cpu().numpy()
    vals = _HDR.unpack(bytes(raw[:_HDR.size]))
    if vals[0] != 0x50524148:
        raise ValueError("save_model: not a model blob (bad magic)")
    hdr = _FILE_HDR.pack(_FILE_MAGIC, _FILE_VERSION, vals[1], _blob_element_hash(raw), raw.size)
    with open(path, "wb") as f:
        f.write(hdr)
        f.write(raw.tobytes())


def load_model(path: str, device="cuda", samples: np.ndarray | None = None,
               wire_radius: float | None = None) -> Model:
    """Read a file written by save_model.  Checks the file magic and version,
    the blob's own magic, version and size, and that the element samples the
    blob carries hash to the recorded element hash; when `samples` (and
    `wire_radius`) are given, also that the file was built from that element.
    Raises ValueError on any mismatch."""
    with open(path, "rb") as f:
        head = f.read(_FILE_HDR.size)
        if len(head) != _FILE_HDR.size:
            raise ValueError(f"load_model: {path}: truncated header")
        magic, fver, bver, ehash, nbytes = _FILE_HDR.unpack(head)
        if magic != _FILE_MAGIC:
            raise ValueError(f"load_model: {path}: not a HARP model file")
        if fver != _FILE_VERSION:
            raise ValueError(f"load_model: {path}: file version {fver}, expected {_FILE_VERSION}")
        raw = np.frombuffer(f.read(), dtype=np.uint8)
    if raw.size != nbytes or raw.size < _HDR.size:
        raise ValueError(f"load_model: {path}: blob of {raw.size} bytes, header says {nbytes}")
    vals = _HDR.unpack(bytes(raw[:_HDR.size]))
    keys = ["magic", "version", "n_mbf", "n_samp", "P", "Q", "n_alpha", "n_t", "freq_hz", "k",
            "omega_mu", "r_min", "wire_radius", "off_coef", "off_coef32", "off_self", "off_port",
            "off_samples", "total_bytes"]
    h = dict(zip(keys, vals))
    if h["magic"] != 0x50524148 or h["version"] != bver or bver != 1:
        raise ValueError(f"load_model: {path}: blob magic / version mismatch")
    if h["total_bytes"] != raw.size or model_layout_bytes(h["n_mbf"], h["n_samp"], h["P"], h["Q"]) != raw.size:
        raise ValueError(f"load_model: {path}: blob size does not match its header")
    if _blob_element_hash(raw) != ehash:
        raise ValueError(f"load_model: {path}: element samples do not match the recorded hash")
    if samples is not None:
        wr = h["wire_radius"] if wire_radius is None else wire_radius
        if element_hash(samples, wr) != ehash:
            raise ValueError(f"load_model: {path}: built from a different element")
    nm, P, Q = h["n_mbf"], h["P"], h["Q"]
    nc = nm * nm * (2 * P + 1) * (Q + 1)
    C = raw[h["off_coef"]:h["off_coef"] + nc * 16].view(np.complex128).reshape(nm, nm, 2 * P + 1, Q + 1)
    Zs = raw[h["off_self"]:h["off_self"] + nm * nm * 16].view(np.complex128).reshape(nm, nm)
    blob = torch.from_numpy(raw.copy()).to(device)
    return Model(blob, nm, h["n_samp"], P, Q, float(h["freq_hz"]), float(h["r_min"]), _table_reciprocal(C, Zs))


def model_layout_bytes(n_mbf: int, n_samp: int, P: int, Q: int) -> int:
    """Size of a model blob (host arithmetic of the layout in include/harp.h;
    equals harp_model_bytes)."""
    def a256(b):
        return (b + 255) & ~255
    ncoef = n_mbf * n_mbf * (2 * P + 1) * (Q + 1)
    return (256 + a256(ncoef * 16) + a256(ncoef * 8) + a256(n_mbf * n_mbf * 16) + a256(n_mbf * 16)
            + a256(n_mbf * n_samp * 8 * 8))


@dataclass
class ModelBatch:
    """Models of one element type at several frequencies, equal stride."""
    data: torch.Tensor      # uint8 [n_freq, stride]
    n_mbf: int
    Q: int
    p_max: int
    freqs: list

    @property
    def n_freq(self) -> int:
        return int(self.data.shape[0])

    @property
    def stride(self) -> int:
        return int(self.data.shape[1])


def stack_models(models) -> ModelBatch:
    n_mbf = {m.n_mbf for m in models}
    Q = {m.Q for m in models}
    if len(n_mbf) != 1 or len(Q) != 1:
        raise ValueError("stack_models: models must share n_mbf and Q")
    stride = max(m.nbytes for m in models)
    stride = (stride + 255) & ~255
    data = torch.zeros((len(models), stride), dtype=torch.uint8, device=models[0].blob.device)
    for i, m in enumerate(models):
        data[i, :m.nbytes] = m.blob
    return ModelBatch(data, n_mbf.pop(), Q.pop(), max(m.P for m in models),
                      [m.freq for m in models])


def read_model_header(model: Model) -> dict:
    vals = _HDR.unpack(bytes(model.blob[:_HDR.size].cpu().numpy()))
    keys = ["magic", "version", "n_mbf", "n_samp", "P", "Q", "n_alpha", "n_t", "freq_hz", "k",
            "omega_mu", "r_min", "wire_radius", "off_coef", "off_coef32", "off_self", "off_port",
            "off_samples", "total_bytes"]
    return dict(zip(keys, vals))


def model_arrays(model: Model) -> dict:
    """Host copies of the sections of a model blob (C, Z_self, w)."""
    h = read_model_header(model)
    raw = model.blob.cpu().numpy()
    nm, P, Q = h["n_mbf"], h["P"], h["Q"]
    nc = nm * nm * (2 * P + 1) * (Q + 1)

    def get(off, n, dt):
        return raw[off:off + n * np.dtype(dt).itemsize].view(dt)

    return {
        "C": get(h["off_coef"], nc, np.complex128).reshape(nm, nm, 2 * P + 1, Q + 1),
        "C32": get(h["off_coef32"], nc, np.complex64).reshape(nm, nm, 2 * P + 1, Q + 1),
        "Z_self": get(h["off_self"], nm * nm, np.complex128).reshape(nm, nm),
        "w": get(h["off_port"], nm, np.complex128),
        "header": h,
    }


# --------------------------------------------------------------------------
# fill, ports
# --------------------------------------------------------------------------

def harp_fill(models: ModelBatch, x: torch.Tensor, y: torch.Tensor, dtype="c64", ri: float = 0.0,
              Z: torch.Tensor | None = None, Z32: torch.Tensor | None = None,
              dual: bool = False, check_domain: bool = True):
    """Fill the reduced matrices of all frequencies (Eq. 4).  Returns (Z, Z32,
    info); with dual=True, Z32 is a second complex64 copy (dtype c128: the
    FP64 result rounded; dtype c64: the same values as Z).
    With check_domain (default) the call waits for the fill and raises
    HARP_E_DOMAIN if a pair is closer than the model's r_min (HARP_E_ARG for a
    model that does not match); otherwise info holds the counts."""
    dt = _DT[dtype]
    dev = models.data.device
    n_ant = int(x.numel())
    n = n_ant * models.n_mbf
    if Z is None:
        Z = colmajor(models.n_freq, n, n, _TORCH_DT[dt], dev)
    if dual and Z32 is None:
        Z32 = colmajor(models.n_freq, n, n, torch.complex64, dev)
    pz, ldz, sz = _cm(Z, "Z")
    p32, ld32, s32 = _cm(Z32, "Z32") if Z32 is not None else (0, 0, 0)
    info = torch.empty(models.n_freq, dtype=torch.int32, device=dev)
    x = x.contiguous()
    y = y.contiguous()
    check(lib().harp_fill(_ptr(models.data), models.stride, models.n_freq, models.n_mbf,
                          models.Q, models.p_max, _ptr(x), _ptr(y), n_ant, float(ri), dt,
                          pz, ldz, sz, p32, ld32, s32, _ptr(info), _stream(dev)), "harp_fill")
    if check_domain:
        check_flags(fill_info=info, where="harp_fill")
    return Z, Z32, info


def harp_port_rhs(models: ModelBatch, n_ant: int, B: torch.Tensor | None = None):
    n = n_ant * models.n_mbf
    dev = models.data.device
    if B is None:
        B = colmajor(models.n_freq, n, n_ant, torch.complex128, dev)
    pb, ldb, sb = _cm(B, "B")
    check(lib().harp_port_rhs(_ptr(models.data), models.stride, models.n_freq, models.n_mbf,
                              n_ant, pb, ldb, sb, _stream(dev)), "harp_port_rhs")
    return B


def harp_port_admittance(models: ModelBatch, X: torch.Tensor, Y: torch.Tensor | None = None):
    n_ant = X.shape[-1]
    dev = models.data.device
    if Y is None:
        Y = colmajor(models.n_freq, n_ant, n_ant, torch.complex128, dev)
    px, ldx, sx = _cm(X, "X")
    py, ldy, sy = _cm(Y, "Y")
    check(lib().harp_port_admittance(_ptr(models.data), models.stride, models.n_freq,
                                     models.n_mbf, n_ant, px, ldx, sx, py, ldy, sy,
                                     _stream(dev)), "harp_port_admittance")
    return Y


# --------------------------------------------------------------------------
# factor, solve
# --------------------------------------------------------------------------

class Factors:
    """LU factors of a batch (in place in `LU`), pivots, info, and the factor
    auxiliary buffer (inverse diagonal blocks, group permutations)."""

    def __init__(self, LU, ipiv, info, aux):
        self.LU, self.ipiv, self.info, self.aux = LU, ipiv, info, aux

    def __iter__(self):            # (ipiv, info) unpacking for convenience
        return iter((self.ipiv, self.info))


def reduced_factor(A: torch.Tensor, check_singular: bool = True) -> Factors:
    """In-place LU with partial pivoting of a batch of column-major matrices.
    With check_singular (default) the call waits for the factorisation and
    raises HARP_E_SINGULAR on an exact zero pivot; otherwise F.info holds the
    pivot indices (LAPACK's info convention)."""
    if A.dim() == 2:
        A = A.unsqueeze(0)
    dt = _DT[A.dtype]
    b, n, _ = A.shape
    pa, lda, sa = _cm(A, "A")
    ipiv = torch.empty((b, n), dtype=torch.int32, device=A.device)
    info = torch.empty(b, dtype=torch.int32, device=A.device)
    ws_b = ctypes.c_size_t()
    check(lib().reduced_factor_ws(n, b, dt, ctypes.byref(ws_b)), "reduced_factor_ws")
    aux = torch.empty(max(1, ws_b.value), dtype=torch.uint8, device=A.device)
    check(lib().reduced_factor(n, b, dt, pa, lda, sa, _ptr(ipiv), _ptr(info), _ptr(aux),
                               ws_b.value, _stream(A.device)), "reduced_factor")
    if check_singular:
        check_flags(factor_info=info, where="reduced_factor")
    return Factors(A, ipiv, info, aux)


def reduced_solve(F: Factors, B: torch.Tensor, X: torch.Tensor | None = None,
                  Z64: torch.Tensor | None = None, tol: float = 1e-12, max_iter: int = 10,
                  raise_noconv: bool = True, device_report: bool = False):
    """Solve with the factors of reduced_factor; optional FP64 refinement
    against Z64 (complex128, or complex64 widened to FP64 in the residual:
    the refinement then converges to that complex64 matrix's solution).
    Returns (X, reports or None).  device_report=True: the
    refinement runs without any host synchronisation (all max_iter sweeps
    enqueued, converged systems skipping them) and the second value is the
    device array of reports (read it with read_reports after the stream)."""
    LU = F.LU
    if B.dim() == 2:
        B = B.unsqueeze(0)
    dt = _DT[LU.dtype]
    b, n, _ = LU.shape
    nrhs = B.shape[-1]
    if X is None:
        X = colmajor(b, n, nrhs, torch.complex128, LU.device)
    pl, lda, sl = _cm(LU, "LU")
    pb, ldb, sb = _cm(B, "B")
    px, ldx, sx = _cm(X, "X")
    ref = None
    rep = None
    rep_dev = None
    if Z64 is not None:
        pz, ldz, sz = _cm(Z64, "Z64")
        if device_report:
            rep_dev = torch.zeros(b * 16, dtype=torch.uint8, device=LU.device)
        if Z64.dtype not in (torch.complex128, torch.complex64):
            raise HarpError(HARP_E_ARG, "reduced_solve: Z64 must be complex128 or complex64")
        ref = HarpRefine(pz, ldz, sz, float(tol), int(max_iter), _ptr(rep_dev),
                         int(Z64.dtype == torch.complex64))
        rep = None if device_report else (HarpRefineReport * b)()
    ws_b = ctypes.c_size_t()
    check(lib().reduced_solve_ws(n, nrhs, b, dt, int(ref is not None), ctypes.byref(ws_b)),
          "reduced_solve_ws")
    ws = torch.empty(max(1, ws_b.value), dtype=torch.uint8, device=LU.device)
    st = lib().reduced_solve(n, nrhs, b, dt, pl, lda, sl, _ptr(F.ipiv), _ptr(F.aux),
                             F.aux.numel(), pb, ldb, sb, px, ldx, sx,
                             ctypes.byref(ref) if ref is not None else None,
                             rep if rep is not None else None, _ptr(ws), ws_b.value,
                             _stream(LU.device))
    X._keep = ws   # the workspace lives until the solution is used
    if st == -4 and not raise_noconv:
        st = 0
    check(st, "reduced_solve")
    if device_report:
        return X, rep_dev
    reports = None
    if rep is not None:
        reports = [{"iters": r.iters, "converged": bool(r.converged), "resid_rel": r.resid_rel}
                   for r in rep]
    return X, reports


def read_reports(rep_dev: torch.Tensor):
    """Refinement reports from a device report array (waits for the stream)."""
    return _reports_from_device(rep_dev)


# --------------------------------------------------------------------------
# patterns
# --------------------------------------------------------------------------

def embedded_patterns(model: Model, x: torch.Tensor, y: torch.Tensor, X: torch.Tensor,
                      theta: torch.Tensor, phi: torch.Tensor) -> torch.Tensor:
    """E[port, dir, (theta, phi)] complex128 for every column of X (Eqs. 5-6)."""
    if X.dim() == 3:
        X = X[0]
    n_ant = int(x.numel())
    n_ports = X.shape[-1]
    n_dir = int(theta.numel())
    px, ldx, _ = _cm(X, "X")
    E = torch.empty((n_ports, n_dir, 2), dtype=torch.complex128, device=X.device)
    ws_b = ctypes.c_size_t()
    check(lib().embedded_patterns_ws(model.n_mbf, n_ant, n_dir, ctypes.byref(ws_b)),
          "embedded_patterns_ws")
    ws = torch.empty(max(1, ws_b.value), dtype=torch.uint8, device=X.device)
    x, y = x.contiguous(), y.contiguous()
    theta, phi = theta.contiguous(), phi.contiguous()
    check(lib().embedded_patterns(_ptr(model.blob), model.n_mbf, _ptr(x), _ptr(y), n_ant, px, ldx,
                                  n_ports, _ptr(theta), _ptr(phi), n_dir, _ptr(E), _ptr(ws),
                                  ws_b.value, _stream(X.device)), "embedded_patterns")
    return E


# --------------------------------------------------------------------------
# adjoint (array synthesis): vector-Jacobian products and an autograd Function
# --------------------------------------------------------------------------

def harp_cgemm(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None, alpha: float = 1.0,
               beta: float = 0.0, D: torch.Tensor | None = None) -> torch.Tensor:
    """D = beta C + alpha A B for batched column-major complex matrices (MFMA)."""
    A3 = A if A.dim() == 3 else A.unsqueeze(0)
    B3 = B if B.dim() == 3 else B.unsqueeze(0)
    b, M, K = A3.shape
    N = B3.shape[-1]
    if D is None:
        D = colmajor(b, M, N, A3.dtype, A3.device)
    pa, lda, sa = _cm(A3, "A")
    pb, ldb, sb = _cm(B3, "B")
    pd, ldd, sd = _cm(D, "D")
    pc, ldc, sc = _cm(C, "C") if C is not None else (0, ldd, sd)
    check(lib().harp_cgemm(_DT[A3.dtype], M, N, K, b, float(alpha), pa, lda, sa, pb, ldb, sb, float(beta),
                           pc, ldc, sc, pd, ldd, sd, _stream(A3.device)), "harp_cgemm")
    return D


def cmatrix_copy(src: torch.Tensor, transpose: bool = False, conj: bool = False) -> torch.Tensor:
    """op(src) for batched column-major complex128 matrices (transpose / conjugate)."""
    S = src if src.dim() == 3 else src.unsqueeze(0)
    b, r, c = S.shape
    dst = colmajor(b, c, r, torch.complex128, S.device) if transpose else colmajor(b, r, c, torch.complex128,
                                                                                     S.device)
    ps, lds, ss = _cm(S, "src")
    pd, ldd, sd = _cm(dst, "dst")
    check(lib().harp_cmatrix_copy(r, c, b, ps, lds, ss, pd, ldd, sd, int(transpose), int(conj),
                                  _stream(S.device)), "harp_cmatrix_copy")
    return dst


def harp_port_admittance_vjp(models: ModelBatch, gY: torch.Tensor) -> torch.Tensor:
    """Cotangent of X through Y = W^T X: gX[(i,T), q] = conj(w_T) gY[i, q]."""
    gY3 = gY if gY.dim() == 3 else gY.unsqueeze(0)
    n_ant = gY3.shape[-1]
    n = n_ant * models.n_mbf
    gX = colmajor(models.n_freq, n, n_ant, torch.complex128, gY3.device)
    py, ldy, sy = _cm(gY3, "gY")
    px, ldx, sx = _cm(gX, "gX")
    check(lib().harp_port_admittance_vjp(_ptr(models.data), models.stride, models.n_freq, models.n_mbf,
                                         n_ant, py, ldy, sy, px, ldx, sx, _stream(gY3.device)),
          "harp_port_admittance_vjp")
    return gX


def harp_fill_vjp(models: ModelBatch, x: torch.Tensor, y: torch.Tensor, W: torch.Tensor, ri: float = 0.0,
                  gx: torch.Tensor | None = None, gy: torch.Tensor | None = None):
    """gx_i += Re sum_ab W_ab dZ_ab/dx_i (and y) for the first model of the batch."""
    n_ant = int(x.numel())
    dev = x.device
    if gx is None:
        gx = torch.zeros(n_ant, dtype=torch.float64, device=dev)
    if gy is None:
        gy = torch.zeros(n_ant, dtype=torch.float64, device=dev)
    pw, ldw, _ = _cm(W, "W")
    ws_b = ctypes.c_size_t()
    check(lib().harp_fill_vjp_ws(n_ant, ctypes.byref(ws_b)), "harp_fill_vjp_ws")
    ws = torch.empty(max(1, ws_b.value), dtype=torch.uint8, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    x, y = x.contiguous(), y.contiguous()
    check(lib().harp_fill_vjp(_ptr(models.data), models.n_mbf, models.Q, _ptr(x), _ptr(y), n_ant, float(ri),
                              pw, ldw, _ptr(gx), _ptr(gy), _ptr(info), _ptr(ws), ws_b.value, _stream(dev)),
          "harp_fill_vjp")
    return gx, gy, info


def embedded_patterns_vjp(model: Model, x: torch.Tensor, y: torch.Tensor, X: torch.Tensor,
                          theta: torch.Tensor, phi: torch.Tensor, gE: torch.Tensor, gX: torch.Tensor,
                          gx: torch.Tensor, gy: torch.Tensor):
    """gX += A^H gE and gx, gy += the explicit position dependence of the patterns."""
    X2 = X[0] if X.dim() == 3 else X
    n_ant = int(x.numel())
    n_ports = X2.shape[-1]
    n_dir = int(theta.numel())
    px, ldx, _ = _cm(X2, "X")
    pg, ldg, _ = _cm(gX[0] if gX.dim() == 3 else gX, "gX")
    gE = gE.contiguous()
    ws_b = ctypes.c_size_t()
    check(lib().embedded_patterns_vjp_ws(model.n_mbf, n_ant, n_dir, n_ports, ctypes.byref(ws_b)),
          "embedded_patterns_vjp_ws")
    ws = torch.empty(max(1, ws_b.value), dtype=torch.uint8, device=X2.device)
    x, y = x.contiguous(), y.contiguous()
    theta, phi = theta.contiguous(), phi.contiguous()
    check(lib().embedded_patterns_vjp(_ptr(model.blob), model.n_mbf, _ptr(x), _ptr(y), n_ant, px, ldx,
                                      n_ports, _ptr(theta), _ptr(phi), n_dir, _ptr(gE), pg, ldg, _ptr(gx),
                                      _ptr(gy), _ptr(ws), ws_b.value, _stream(X2.device)),
          "embedded_patterns_vjp")


class ArrayResponse(torch.autograd.Function):
    """(x, y) -> (Y, E): port admittances (n_ant x n_ant) and embedded element
    patterns ([port][dir][theta/phi]) of one element type at one frequency,
    through the Eq. 4 fill (complex128), a complex128 LU solve with one
    right-hand side per port, and Eqs. 5-6.  The backward pass is the
    hand-written adjoint: the patterns' and ports' vector-Jacobian products,
    one adjoint solve with the same factors (Z is complex-symmetric), the
    cotangent of Z as the product -conj(Lambda) X^T, and the fill's product.
    The forward pass raises HARP_E_DOMAIN for a pair closer than the model's
    r_min (e.g. an optimiser step that brings two elements too close) and
    HARP_E_SINGULAR for an exact zero pivot."""

    @staticmethod
    def forward(ctx, x, y, model, theta, phi, ri):
        if not model.reciprocal:
            raise ValueError("array_response: the adjoint solves with Z instead of Z^T, which needs a "
                             "reciprocal model table (C^{ST}_p = (-1)^p C^{TS}_p, symmetric self block)")
        mb = stack_models([model])
        x64 = x.detach().to(torch.float64).contiguous()
        y64 = y.detach().to(torch.float64).contiguous()
        Z, _, info = harp_fill(mb, x64, y64, dtype="c128", ri=ri)
        F = reduced_factor(Z)
        B = harp_port_rhs(mb, int(x64.numel()))
        X, _ = reduced_solve(F, B)
        Y = harp_port_admittance(mb, X)
        E = embedded_patterns(model, x64, y64, X, theta, phi)
        ctx.save_for_backward(x64, y64, theta, phi)
        ctx.F, ctx.X, ctx.mb, ctx.model, ctx.ri, ctx.info, ctx.finfo = F, X, mb, model, ri, info, F.info
        return Y[0], E

    @staticmethod
    def backward(ctx, gY, gE):
        x, y, theta, phi = ctx.saved_tensors
        dev = x.device
        n_ant = int(x.numel())
        gx = torch.zeros(n_ant, dtype=torch.float64, device=dev)
        gy = torch.zeros(n_ant, dtype=torch.float64, device=dev)
        X = ctx.X
        if gY is None:
            gY = torch.zeros((n_ant, n_ant), dtype=torch.complex128, device=dev)
        gX = harp_port_admittance_vjp(ctx.mb, gY.resolve_conj().transpose(0, 1).contiguous().transpose(0, 1))
        if gE is not None:
            embedded_patterns_vjp(ctx.model, x, y, X, theta, phi, gE.resolve_conj(), gX, gx, gy)
        # Lambda = Z^-H gX = conj(Z^-1 conj(gX));  W = -conj(Lambda) X^T = -(Z^-1 conj(gX)) X^T
        Lc, _ = reduced_solve(ctx.F, cmatrix_copy(gX, conj=True))
        W = harp_cgemm(Lc, cmatrix_copy(X, transpose=True), alpha=-1.0)
        harp_fill_vjp(ctx.mb, x, y, W, ri=ctx.ri, gx=gx, gy=gy)
        return gx, gy, None, None, None, None


def array_response(x: torch.Tensor, y: torch.Tensor, model: Model, theta: torch.Tensor, phi: torch.Tensor,
                   ri: float = 0.0):
    """Differentiable (Y, E) of a layout; see ArrayResponse."""
    return ArrayResponse.apply(x, y, model, theta, phi, ri)


def to_device_samples(samples: np.ndarray, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(samples, dtype=np.float64)).to(device)


def default_grid(P: int, Q: int):
    return 4 * (P + 1), 2 * (Q + 1)


__all__ = [
    "Model", "ModelBatch", "harp_fit", "pack_model", "stack_models", "harp_fill",
    "harp_port_rhs", "harp_port_admittance", "reduced_factor", "reduced_solve", "Factors",
    "embedded_patterns", "colmajor", "model_bytes", "model_arrays", "read_model_header",
    "to_device_samples", "default_grid", "harp_cgemm", "cmatrix_copy", "harp_port_admittance_vjp",
    "harp_fill_vjp", "embedded_patterns_vjp", "ArrayResponse", "array_response",
    "save_model", "load_model", "read_reports", "set_tuning", "get_tuning", "default_tuning",
    "autotune_kernels", "element_hash", "check_flags", "HarpError",
    "SYSTEM_DTYPE", "systems_tensor", "harp_batch_plan", "autotune_batch_costs", "harp_fill_systems", "harp_port_rhs_systems",
    "harp_port_admittance_systems", "BatchSolver", "StationSolver", "Cell", "harp_tessellate",
    "TessellatedSolver",
]


# --------------------------------------------------------------------------
# whole hot path with preallocated buffers
# --------------------------------------------------------------------------

class StationSolver:
    """Fill, factor, port excitation, solve and admittances for a batch of
    frequencies of one layout, with every device buffer allocated once.

    mode "refined": FP64 fill written as complex128 (residual matrix) and as
    its complex64 rounding (factored on the matrix cores), complex64 solve,
    FP64 iterative refinement to `tol` (convergence decided on the device;
    the host waits once, after the first correction, in the common case).
    mode "refined32": complex64 fill (FP32 evaluation, FP64 phase argument)
    written twice, one copy factored on the matrix cores and the other kept
    as the matrix of the FP64 residual (widened as it is read); the
    refinement converges to the complex64 matrix's solution.
    mode "plain": complex128 fill, factor and solve (the FP64 reference path).
    ri > 0: radius of influence of the fill (blocks of pairs farther apart are
    zero, Section II-D).
    """

    def __init__(self, models: ModelBatch, x: torch.Tensor, y: torch.Tensor, mode="refined",
                 tol: float = 1e-10, max_iter: int = 10, ri: float = 0.0, host_report: bool = True):
        self.models, self.mode, self.tol, self.max_iter, self.ri = models, mode, tol, max_iter, float(ri)
        # host_report=False: the refinement never synchronises (its report stays
        # on the device; every one of the max_iter sweeps is enqueued)
        self.host_report = host_report
        dev = models.data.device
        self.x = x.contiguous()
        self.y = y.contiguous()
        self.n_ant = int(x.numel())
        n = self.n = self.n_ant * models.n_mbf
        nf = models.n_freq
        if mode not in ("refined", "refined32", "plain"):
            raise ValueError(f"StationSolver: unknown mode {mode!r}")
        self.refined = mode != "plain"
        # the matrix of the residual (refined modes) or the factored one (plain)
        self.Z64 = colmajor(nf, n, n, torch.complex128, dev) if mode != "refined32" else None
        self.Zr = colmajor(nf, n, n, torch.complex64, dev) if mode == "refined32" else None
        self.Z32 = colmajor(nf, n, n, torch.complex64, dev) if self.refined else None
        self.B = colmajor(nf, n, self.n_ant, torch.complex128, dev)
        self.X = colmajor(nf, n, self.n_ant, torch.complex128, dev)
        self.Y = colmajor(nf, self.n_ant, self.n_ant, torch.complex128, dev)
        # fill domain counts (row 0) and zero-pivot indices (row 1), read together
        self.flags = torch.zeros((2, nf), dtype=torch.int32, device=dev)
        self.info, self.finfo = self.flags[0], self.flags[1]
        self.ipiv = torch.empty((nf, n), dtype=torch.int32, device=dev)
        dt = C64 if self.refined else C128
        aux_b = ctypes.c_size_t()
        check(lib().reduced_factor_ws(n, nf, dt, ctypes.byref(aux_b)), "reduced_factor_ws")
        self.aux = torch.empty(max(1, aux_b.value), dtype=torch.uint8, device=dev)
        self.aux_bytes = aux_b.value
        ws_b = ctypes.c_size_t()
        check(lib().reduced_solve_ws(n, self.n_ant, nf, dt, int(self.refined),
                                     ctypes.byref(ws_b)), "reduced_solve_ws")
        self.ws = torch.empty(max(1, ws_b.value), dtype=torch.uint8, device=dev)
        self.ws_bytes = ws_b.value
        self.rep_dev = torch.zeros(nf * 16, dtype=torch.uint8, device=dev)
        self._reports = None

    @property
    def reports(self):
        """Refinement report per frequency (read from the device)."""
        if not self.refined:
            return None
        if self._reports is None:
            self._reports = _reports_from_device(self.rep_dev)
        return self._reports

    def step(self, events=None, check_flags_: bool = True):
        """One pass of the hot path.  events: optional five torch.cuda.Event
        recorded on the stream at the phase boundaries (start, after fill and
        excitation, after the factorisation, after the solve and refinement,
        after the admittances).  With check_flags_ (default) the fill's domain
        counts and the factorisation's zero pivots are read at the end and
        raised (HARP_E_DOMAIN, HARP_E_SINGULAR)."""
        L = lib()
        mb, n, na, nf = self.models, self.n, self.n_ant, self.models.n_freq
        st = _stream(mb.data.device)
        refined = self.refined
        z32 = self.mode == "refined32"
        mark = (lambda i: events[i].record()) if events is not None else (lambda i: None)
        mark(0)
        pz, ldz, sz = _cm(self.Zr, "Zr") if z32 else _cm(self.Z64, "Z64")
        p32, ld32, s32 = _cm(self.Z32, "Z32") if refined else (0, 0, 0)
        check(L.harp_fill(_ptr(mb.data), mb.stride, nf, mb.n_mbf, mb.Q, mb.p_max, _ptr(self.x),
                          _ptr(self.y), na, self.ri, C64 if z32 else C128, pz, ldz, sz, p32, ld32, s32,
                          _ptr(self.info), st), "harp_fill")
        pb, ldb, sb = _cm(self.B, "B")
        check(L.harp_port_rhs(_ptr(mb.data), mb.stride, nf, mb.n_mbf, na, pb, ldb, sb, st),
              "harp_port_rhs")
        mark(1)
        pf, ldf, sf = (p32, ld32, s32) if refined else (pz, ldz, sz)
        dt = C64 if refined else C128
        check(L.reduced_factor(n, nf, dt, pf, ldf, sf, _ptr(self.ipiv), _ptr(self.finfo),
                               _ptr(self.aux), self.aux_bytes, st), "reduced_factor")
        mark(2)
        px, ldx, sx = _cm(self.X, "X")
        ref = HarpRefine(pz, ldz, sz, float(self.tol), int(self.max_iter), _ptr(self.rep_dev),
                         int(z32)) if refined else None
        rep = (HarpRefineReport * nf)() if (refined and self.host_report) else None
        self._reports = None
        status = L.reduced_solve(n, na, nf, dt, pf, ldf, sf, _ptr(self.ipiv), _ptr(self.aux),
                                 self.aux_bytes, pb, ldb, sb, px, ldx,
                                 sx, ctypes.byref(ref) if ref is not None else None, rep,
                                 _ptr(self.ws), self.ws_bytes, st)
        if status not in (0, -4):          # argument / workspace / runtime errors: nothing more to enqueue
            check(status, "reduced_solve")
        mark(3)
        py, ldy, sy = _cm(self.Y, "Y")
        check(L.harp_port_admittance(_ptr(mb.data), mb.stride, nf, mb.n_mbf, na, px, ldx, sx, py,
                                     ldy, sy, st), "harp_port_admittance")
        mark(4)
        if check_flags_:
            fl = self.flags.cpu().numpy()
            check_flags(fl[0], fl[1], "StationSolver.step")
        check(status, "reduced_solve")
        return self.X, self.Y


# --------------------------------------------------------------------------
# batches of unequal layouts
# --------------------------------------------------------------------------

SYSTEM_DTYPE = np.dtype([("model", "<i4"), ("n_ant", "<i4"), ("pos", "<i8"), ("n_ports", "<i4"),
                         ("reserved", "<i4")])   # harp_system


def systems_tensor(model_idx, n_ant, pos, device="cuda", n_ports=None) -> torch.Tensor:
    """Device array of harp_system descriptors (24 bytes each); n_ports None
    or 0: every antenna of a system is a port."""
    a = np.zeros(len(model_idx), dtype=SYSTEM_DTYPE)
    a["model"], a["n_ant"], a["pos"] = model_idx, n_ant, pos
    if n_ports is not None:
        a["n_ports"] = n_ports
    return torch.from_numpy(a.view(np.uint8).copy()).to(device)


def harp_batch_plan(n_ant, n_mbf: int, pad_multiple: int = 8, max_order: int = 8192,
                    max_batch: int = 96, cost=None):
    """Grouping of unequal systems: (order, groups), groups = [(begin, end,
    n_ant_pad)] indexing `order` (system indices sorted by size)."""
    n = len(n_ant)
    na = (ctypes.c_int32 * n)(*[int(v) for v in n_ant])
    order = (ctypes.c_int32 * n)()
    gb = (ctypes.c_int32 * (n + 1))()
    gp = (ctypes.c_int32 * n)()
    ng = ctypes.c_int32()
    c = (ctypes.c_double * 3)(*cost) if cost is not None else None
    check(lib().harp_batch_plan(na, n, n_mbf, pad_multiple, max_order, max_batch, c, order, gb, gp,
                                ctypes.byref(ng)), "harp_batch_plan")
    groups = [(gb[g], gb[g + 1], gp[g]) for g in range(ng.value)]
    return list(order), groups


def harp_fill_systems(models: ModelBatch, x: torch.Tensor, y: torch.Tensor, sys: torch.Tensor,
                      n_ant_pad: int, dtype="c128", ri: float = 0.0, Z: torch.Tensor | None = None,
                      Z32: torch.Tensor | None = None, dual: bool = False, check_domain: bool = True):
    """Fill a group of systems padded to n_ant_pad antennas.  Returns (Z, Z32,
    info); check_domain as for harp_fill."""
    dt = _DT[dtype]
    dev = models.data.device
    n_sys = sys.numel() // SYSTEM_DTYPE.itemsize
    n = n_ant_pad * models.n_mbf
    if Z is None:
        Z = colmajor(n_sys, n, n, _TORCH_DT[dt], dev)
    if dual and Z32 is None:
        Z32 = colmajor(n_sys, n, n, torch.complex64, dev)
    pz, ldz, sz = _cm(Z, "Z")
    p32, ld32, s32 = _cm(Z32, "Z32") if Z32 is not None else (0, 0, 0)
    info = torch.empty(n_sys, dtype=torch.int32, device=dev)
    x, y = x.contiguous(), y.contiguous()
    check(lib().harp_fill_systems(_ptr(models.data), models.stride, models.n_freq, models.n_mbf, models.Q,
                                  models.p_max, _ptr(x), _ptr(y), int(x.numel()), _ptr(sys), n_sys, n_ant_pad,
                                  float(ri), dt, pz, ldz, sz, p32, ld32, s32, _ptr(info), _stream(dev)),
          "harp_fill_systems")
    if check_domain:
        check_flags(fill_info=info, where="harp_fill_systems")
    return Z, Z32, info


def harp_port_rhs_systems(models: ModelBatch, sys: torch.Tensor, n_ant_pad: int,
                          n_ports_pad: int | None = None, B: torch.Tensor | None = None):
    dev = models.data.device
    n_sys = sys.numel() // SYSTEM_DTYPE.itemsize
    n = n_ant_pad * models.n_mbf
    n_ports_pad = n_ant_pad if n_ports_pad is None else n_ports_pad
    if B is None:
        B = colmajor(n_sys, n, n_ports_pad, torch.complex128, dev)
    pb, ldb, sb = _cm(B, "B")
    check(lib().harp_port_rhs_systems(_ptr(models.data), models.stride, models.n_freq, models.n_mbf, _ptr(sys),
                                      n_sys, n_ant_pad, n_ports_pad, pb, ldb, sb, _stream(dev)),
          "harp_port_rhs_systems")
    return B


def harp_port_admittance_systems(models: ModelBatch, sys: torch.Tensor, X: torch.Tensor,
                                 Y: torch.Tensor | None = None):
    """Y_s = W^T X_s (n_ant_pad x n_ports_pad) for X (n_sys, N, n_ports_pad)."""
    dev = models.data.device
    n_sys = sys.numel() // SYSTEM_DTYPE.itemsize
    n_ant_pad = X.shape[-2] // models.n_mbf
    n_ports_pad = X.shape[-1]
    if Y is None:
        Y = colmajor(n_sys, n_ant_pad, n_ports_pad, torch.complex128, dev)
    px, ldx, sx = _cm(X, "X")
    py, ldy, sy = _cm(Y, "Y")
    check(lib().harp_port_admittance_systems(_ptr(models.data), models.stride, models.n_freq, models.n_mbf,
                                             _ptr(sys), n_sys, n_ant_pad, n_ports_pad, px, ldx, sx, py, ldy, sy,
                                             _stream(dev)), "harp_port_admittance_systems")
    return Y


class _Group:
    """Device buffers of one padded group (refined path).  info / finfo are
    views into the batch's shared flag array.  Zres is the matrix of the FP64
    residual: complex128 (FP64 fill) or complex64 (complex64 fill, the second
    copy of the fill); Z32 is the copy that is factored."""

    def __init__(self, models: ModelBatch, members, n_pad, model_idx, n_ant, pos, n_ports, pad_multiple, dev,
                 flags, off, fill32=False):
        self.members, self.n_pad = members, n_pad
        c = len(members)
        n = self.n = n_pad * models.n_mbf
        npmax = max(n_ports[i] for i in members)
        self.n_ports_pad = min(n_pad, -(-npmax // pad_multiple) * pad_multiple)
        self.sys = systems_tensor([model_idx[i] for i in members], [n_ant[i] for i in members],
                                  [pos[i] for i in members], dev, n_ports=[n_ports[i] for i in members])
        npp = self.n_ports_pad
        self.fill32 = fill32
        self.Zres = colmajor(c, n, n, torch.complex64 if fill32 else torch.complex128, dev)
        self.Z64 = None if fill32 else self.Zres
        self.Z32 = colmajor(c, n, n, torch.complex64, dev)
        self.B = colmajor(c, n, npp, torch.complex128, dev)
        self.X = colmajor(c, n, npp, torch.complex128, dev)
        self.Y = colmajor(c, n_pad, npp, torch.complex128, dev)
        self.info = flags[0, off:off + c]
        self.finfo = flags[1, off:off + c]
        self.ipiv = torch.empty((c, n), dtype=torch.int32, device=dev)
        # refinement report on the device (harp_refine_report, 16 bytes each)
        self.rep_dev = torch.zeros(c * 16, dtype=torch.uint8, device=dev)
        b = ctypes.c_size_t()
        check(lib().reduced_factor_ws(n, c, C64, ctypes.byref(b)), "reduced_factor_ws")
        self.aux, self.aux_bytes = torch.empty(max(1, b.value), dtype=torch.uint8, device=dev), b.value
        check(lib().reduced_solve_ws(n, npp, c, C64, 1, ctypes.byref(b)), "reduced_solve_ws")
        self.ws, self.ws_bytes = torch.empty(max(1, b.value), dtype=torch.uint8, device=dev), b.value


_REPORT_DTYPE = np.dtype([("iters", "<i4"), ("converged", "<i4"), ("resid_rel", "<f8")])


def _reports_from_device(rep_dev: torch.Tensor):
    a = rep_dev.cpu().numpy().view(_REPORT_DTYPE)
    return [{"iters": int(r["iters"]), "converged": bool(r["converged"]), "resid_rel": float(r["resid_rel"])}
            for r in a]


def autotune_batch_costs(models: ModelBatch, sizes=(96, 256, 480), counts=(1, 8), reps: int = 2,
                         seed: int = 7, tol: float = 1e-10):
    """Measure the batch path on this GPU and fit the planner's cost model
    t(group) = t_group + t_order N + t_system c N^3 (N = padded order, c
    systems): one group of c systems of n_ant antennas (seeded random layouts
    at the station density, model 0) per (n_ant, c) pair, timed over `reps`
    passes after one warm-up, then a non-negative least-squares fit.  Returns
    (cost triple for harp_batch_plan, the measured points)."""
    from scipy.optimize import nnls
    rng = np.random.default_rng(seed)
    rows, times, points = [], [], []
    for na in sizes:
        # random sequential addition in a disk of the station density
        radius = 19.0 * math.sqrt(na / 256.0)
        pts = []
        while len(pts) < na:
            u, v = rng.uniform(size=2)
            px, py = radius * math.sqrt(u) * math.cos(2 * math.pi * v), radius * math.sqrt(u) * math.sin(2 * math.pi * v)
            if all((px - a) ** 2 + (py - b) ** 2 >= 1.5 ** 2 for a, b in pts):
                pts.append((px, py))
        x, y = np.array(pts).T
        for c in counts:
            S = BatchSolver(models, [(x, y, [0] * c)], tol=tol, streams=1, max_batch=c, pad_multiple=8,
                            cost=[1.0, 0.0, 0.0])
            S.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                S.step()
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            N = float(S.groups[0].n)
            rows.append([1.0, N, c * N ** 3])
            times.append(t)
            points.append({"n_ant": int(na), "systems": int(c), "order": int(N), "seconds": t})
            del S
    A = np.array(rows)
    scale = A.max(axis=0)
    coef, _ = nnls(A / scale, np.array(times))
    return [float(v) for v in coef / scale], points


# --------------------------------------------------------------------------
# kernel tuning per matrix order
# --------------------------------------------------------------------------

def set_tuning(entries) -> None:
    """Install a kernel tuning table (list of dicts with max_order,
    panel_width_c64, panel_width_c128, small_grid_wgs; ascending max_order);
    None or [] restores the built-in choices."""
    entries = entries or []
    arr = (HarpTuningEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i] = HarpTuningEntry(int(e["max_order"]), int(e["panel_width_c64"]), int(e["panel_width_c128"]),
                                 int(e["small_grid_wgs"]))
    check(lib().harp_set_tuning(arr, len(entries)), "harp_set_tuning")


def get_tuning() -> list:
    arr = (HarpTuningEntry * 64)()
    n = ctypes.c_int32()
    check(lib().harp_get_tuning(arr, 64, ctypes.byref(n)), "harp_get_tuning")
    return [{"max_order": e.max_order, "panel_width_c64": e.panel_width_c64,
             "panel_width_c128": e.panel_width_c128, "small_grid_wgs": e.small_grid_wgs} for e in arr[:n.value]]


def default_tuning(n: int) -> dict:
    e = HarpTuningEntry()
    check(lib().harp_default_tuning(int(n), ctypes.byref(e)), "harp_default_tuning")
    return {"max_order": e.max_order, "panel_width_c64": e.panel_width_c64,
            "panel_width_c128": e.panel_width_c128, "small_grid_wgs": e.small_grid_wgs}


def autotune_kernels(groups, reps: int = 2, seed: int = 11, widths=(16, 8, 4), small_grids=(256, 1024, 4096),
                     device="cuda"):
    """Pick, for each (order N, systems c, right-hand sides r) in `groups`,
    the complex64 panel width and the GEMM small-grid switch that make a
    complex64 factorisation of c diagonally dominant random systems of order
    N plus one solve with r right-hand sides fastest on this GPU (each
    candidate timed over `reps` passes after one warm-up).  Returns (tuning
    entries for set_tuning / BatchSolver, the measured points).  The table in
    force when the call started is restored."""
    saved = get_tuning()
    rng = np.random.default_rng(seed)
    entries, points = [], []
    try:
        for N, c, r in sorted(set((int(a), int(b), int(d)) for a, b, d in groups)):
            A = rng.standard_normal((c, N, N)) + 1j * rng.standard_normal((c, N, N))
            A += 3.0 * math.sqrt(N) * np.eye(N)[None]
            A0 = colmajor(c, N, N, torch.complex64, device)
            A0.copy_(torch.from_numpy(A.astype(np.complex64)))
            B = colmajor(c, N, r, torch.complex128, device)
            B.copy_(torch.from_numpy(rng.standard_normal((c, N, r)) + 0j))
            W = colmajor(c, N, N, torch.complex64, device)
            base = default_tuning(N)
            best = None
            for w in widths:
                for sg in small_grids:
                    e = dict(base, panel_width_c64=w, small_grid_wgs=sg)
                    try:
                        set_tuning([e])
                    except HarpError:
                        continue          # no launch configuration for this width at this order
                    times = []
                    for it in range(reps + 1):
                        W.copy_(A0)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        F = reduced_factor(W, check_singular=False)
                        reduced_solve(F, B)
                        torch.cuda.synchronize()
                        if it:
                            times.append(time.perf_counter() - t0)
                    t = min(times)
                    points.append({"order": N, "systems": c, "rhs": r, "panel_width_c64": w,
                                   "small_grid_wgs": sg, "seconds": t})
                    if best is None or t < best[0]:
                        best = (t, e)
            entries.append(dict(best[1], max_order=N))
            del A0, B, W
    finally:
        set_tuning(saved)
    return entries, points


class BatchSolver:
    """The refined hot path (fill, complex64 LU, solve, FP64 refinement,
    admittances) for a batch of unequal layouts, each at several
    frequencies, reusing one model per frequency.  fill="c128": FP64 fill
    written as complex128 (the residual's matrix) and complex64 (factored);
    fill="c64": complex64 fill written twice, the FP64 residual taken against
    one copy (widened as it is read).  A layout is (x, y, frequency indices) or (x, y, frequency
    indices, n_ports): its ports are its first n_ports antennas (default all).
    Systems are grouped by harp_batch_plan and padded per group; groups are
    issued round-robin on `streams` HIP streams (default priority), all
    buffers allocated once.  tuning: kernel tuning entries (autotune_kernels)
    installed before the work is enqueued.

    graph=False: each group's refinement reports to the host (one
    synchronisation per group in the common case).  graph=True: the whole
    step -- every group's fill, excitation, factorisation, solve with a
    device-controlled refinement of at most `sweeps` corrections, and
    admittances -- is captured once as one HIP graph and replayed; nothing
    synchronises inside a step and the reports are read from the device."""

    def __init__(self, models: ModelBatch, layouts, tol: float = 1e-10, max_iter: int = 10,
                 streams: int = 1, ri: float = 0.0, graph: bool = False, sweeps: int = 3, tuning=None,
                 fill: str = "c128", **plan_kw):
        if fill not in ("c128", "c64"):
            raise ValueError(f"BatchSolver: fill must be 'c128' or 'c64', not {fill!r}")
        self.fill32 = fill == "c64"
        dev = models.data.device
        self.models, self.tol, self.max_iter, self.ri = models, tol, max_iter, ri
        self.tuning = tuning
        self.graph_mode, self.sweeps = graph, sweeps
        xs, ys, model_idx, n_ant, pos, n_ports, self.layout_of = [], [], [], [], [], [], []
        off = 0
        for li, lay in enumerate(layouts):
            x, y, fidx = lay[0], lay[1], lay[2]
            xs.append(np.asarray(x, dtype=np.float64))
            ys.append(np.asarray(y, dtype=np.float64))
            npt = int(lay[3]) if len(lay) > 3 else int(xs[-1].size)
            if not 0 < npt <= xs[-1].size:
                raise ValueError(f"layout {li}: n_ports {npt} not in [1, {xs[-1].size}]")
            for f in fidx:
                model_idx.append(int(f))
                n_ant.append(int(xs[-1].size))
                n_ports.append(npt)
                pos.append(off)
                self.layout_of.append((li, int(f)))
            off += xs[-1].size
        self.x = torch.from_numpy(np.concatenate(xs)).to(dev)
        self.y = torch.from_numpy(np.concatenate(ys)).to(dev)
        self.n_ant, self.n_ports = n_ant, n_ports
        order, groups = harp_batch_plan(n_ant, models.n_mbf, **plan_kw)
        pm = plan_kw.get("pad_multiple", 8)
        self.flags = torch.zeros((2, len(n_ant)), dtype=torch.int32, device=dev)
        self.groups = []
        for b, e, pad in groups:
            self.groups.append(_Group(models, order[b:e], pad, model_idx, n_ant, pos, n_ports, pm, dev,
                                      self.flags, b, fill32=self.fill32))
        self.where = {}
        for gi, g in enumerate(self.groups):
            for k, s in enumerate(g.members):
                self.where[s] = (gi, k)
        self.streams = [torch.cuda.Stream(dev) for _ in range(streams - 1)]
        self._reports = None
        self._graph = None

    @property
    def n_systems(self) -> int:
        return len(self.n_ant)

    def _front(self, g: _Group, st: int):
        L, mb = lib(), self.models
        c = len(g.members)
        pz, ldz, sz = _cm(g.Zres, "Zres")
        p32, ld32, s32 = _cm(g.Z32, "Z32")
        check(L.harp_fill_systems(_ptr(mb.data), mb.stride, mb.n_freq, mb.n_mbf, mb.Q, mb.p_max, _ptr(self.x),
                                  _ptr(self.y), int(self.x.numel()), _ptr(g.sys), c, g.n_pad, float(self.ri),
                                  C64 if g.fill32 else C128, pz, ldz, sz, p32, ld32, s32, _ptr(g.info), st),
              "harp_fill_systems")
        pb, ldb, sb = _cm(g.B, "B")
        check(L.harp_port_rhs_systems(_ptr(mb.data), mb.stride, mb.n_freq, mb.n_mbf, _ptr(g.sys), c, g.n_pad,
                                      g.n_ports_pad, pb, ldb, sb, st), "harp_port_rhs_systems")
        check(L.reduced_factor(g.n, c, C64, p32, ld32, s32, _ptr(g.ipiv), _ptr(g.finfo), _ptr(g.aux),
                               g.aux_bytes, st), "reduced_factor")

    def _back(self, g: _Group, st: int, host: bool):
        L, mb = lib(), self.models
        c = len(g.members)
        pz, ldz, sz = _cm(g.Zres, "Zres")
        p32, ld32, s32 = _cm(g.Z32, "Z32")
        pb, ldb, sb = _cm(g.B, "B")
        px, ldx, sx = _cm(g.X, "X")
        ref = HarpRefine(pz, ldz, sz, float(self.tol), int(self.max_iter if host else self.sweeps),
                         _ptr(g.rep_dev), int(g.fill32))
        rep = (HarpRefineReport * c)() if host else None
        status = L.reduced_solve(g.n, g.n_ports_pad, c, C64, p32, ld32, s32, _ptr(g.ipiv), _ptr(g.aux),
                                 g.aux_bytes, pb, ldb, sb, px, ldx, sx, ctypes.byref(ref), rep, _ptr(g.ws),
                                 g.ws_bytes, st)
        if status not in (0, -4):
            check(status, "reduced_solve")
        py, ldy, sy = _cm(g.Y, "Y")
        check(L.harp_port_admittance_systems(_ptr(mb.data), mb.stride, mb.n_freq, mb.n_mbf, _ptr(g.sys), c,
                                             g.n_pad, g.n_ports_pad, px, ldx, sx, py, ldy, sy, st),
              "harp_port_admittance_systems")
        return status

    def _enqueue(self, host: bool):
        """Every group's work on the current stream and the side streams
        (forked from and joined back into the current stream), under the
        solver's kernel tuning table (if any)."""
        if self.tuning is not None:
            set_tuning(self.tuning)
        main = torch.cuda.current_stream(self.models.data.device)
        sts = [main] + self.streams
        for s in self.streams:
            s.wait_stream(main)
        for gi, g in enumerate(self.groups):
            self._front(g, sts[gi % len(sts)].cuda_stream)
        noconv = False
        for gi, g in enumerate(self.groups):
            noconv |= self._back(g, sts[gi % len(sts)].cuda_stream, host) == -4
        for s in self.streams:
            main.wait_stream(s)
        return noconv

    def step(self, check_flags_: bool = True):
        """One pass over every system.  Fill, excitation and factorisation of
        all groups are enqueued first, then the solves and admittances.  With
        check_flags_ (default) the domain counts and zero pivots of every
        system are read at the end and raised (HARP_E_DOMAIN,
        HARP_E_SINGULAR)."""
        self._reports = None
        if self.graph_mode:
            if self._graph is None:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    self._enqueue(host=False)
                self._graph = g
            self._graph.replay()
            noconv = False
        else:
            noconv = self._enqueue(host=True)
        if check_flags_:
            fl = self.flags.cpu().numpy()
            check_flags(fl[0], fl[1], "BatchSolver.step")
        if noconv:
            raise HarpError(-4, "BatchSolver.step: refinement did not converge")

    @property
    def reports(self):
        """Refinement report of every system (read from the device)."""
        if self._reports is None:
            reports = [None] * self.n_systems
            for g in self.groups:
                for k, r in enumerate(_reports_from_device(g.rep_dev)):
                    reports[g.members[k]] = r
            self._reports = reports
        return self._reports

    def system(self, s: int):
        """(X, Y, fill info, factor info) of system s, unpadded views: X is
        n x n_ports, Y is n_ant x n_ports."""
        gi, k = self.where[s]
        g = self.groups[gi]
        na, npt = self.n_ant[s], self.n_ports[s]
        n = na * self.models.n_mbf
        return g.X[k, :n, :npt], g.Y[k, :na, :npt], g.info[k], g.finfo[k]

    def padded(self, s: int):
        """(Zres, X, Y) of system s with its padding; Zres is the matrix of the
        FP64 residual (complex128, or complex64 with fill="c64")."""
        gi, k = self.where[s]
        g = self.groups[gi]
        return g.Zres[k], g.X[k], g.Y[k]


@dataclass
class Cell:
    """One cell of the overlapping-subarray tessellation."""
    center: tuple
    members: np.ndarray     # antenna indices, inner ones first
    n_inner: int


def harp_tessellate(x, y, r_in: float, r_ext: float, origin=(0.0, 0.0)):
    """Cells of the hexagonal overlapping-subarray tessellation (Section II-D)
    of the layout (x, y) (host arrays), see include/harp.h."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = int(x.size)
    dp = ctypes.POINTER(ctypes.c_double)
    nc, nm = ctypes.c_int32(), ctypes.c_int64()
    args = (x.ctypes.data_as(dp), y.ctypes.data_as(dp), n, float(r_in), float(r_ext), float(origin[0]),
            float(origin[1]), ctypes.byref(nc), ctypes.byref(nm))
    check(lib().harp_tessellate(*args, None, None, None, None), "harp_tessellate")
    begin = np.zeros(nc.value + 1, dtype=np.int64)
    inner = np.zeros(nc.value, dtype=np.int32)
    members = np.zeros(max(1, nm.value), dtype=np.int32)
    centers = np.zeros(2 * nc.value, dtype=np.float64)
    check(lib().harp_tessellate(*args, begin.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                inner.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                members.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                centers.ctypes.data_as(dp)), "harp_tessellate")
    return [Cell((float(centers[2 * c]), float(centers[2 * c + 1])), members[begin[c]:begin[c + 1]].copy(),
                 int(inner[c])) for c in range(nc.value)]


class TessellatedSolver:
    """The tessellation approach of Section II-D on the batch path: every
    cell's subarray (its antennas within the outer hexagon, the cell's own
    antennas first) is one system at each frequency, with only the cell's own
    antennas' ports excited; antenna a's solution is taken from its own cell's
    subarray (currents on the subarray's antennas, zero elsewhere)."""

    def __init__(self, models: ModelBatch, x, y, fidx, r_in: float, r_ext: float, origin=(0.0, 0.0),
                 tol: float = 1e-10, max_iter: int = 10, streams: int = 2, **plan_kw):
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        self.fidx = [int(f) for f in fidx]
        self.cells = harp_tessellate(self.x, self.y, r_in, r_ext, origin)
        layouts = [(self.x[c.members], self.y[c.members], self.fidx, c.n_inner) for c in self.cells]
        self.batch = BatchSolver(models, layouts, tol=tol, max_iter=max_iter, streams=streams, **plan_kw)
        self.models = models
        self.cell_of = np.empty(self.x.size, dtype=np.int64)
        self.local = np.empty(self.x.size, dtype=np.int64)
        for ci, c in enumerate(self.cells):
            self.cell_of[c.members[:c.n_inner]] = ci
            self.local[c.members[:c.n_inner]] = np.arange(c.n_inner)

    def step(self):
        self.batch.step()

    def system(self, cell: int, f: int) -> int:
        """Batch system index of (cell, model index f)."""
        return cell * len(self.fidx) + self.fidx.index(int(f))

    def port(self, a: int, f: int):
        """(subarray antenna indices, X column (n_sub N_m), Y column (n_sub))
        of a unit voltage at port a at model index f."""
        ci = int(self.cell_of[a])
        X, Y, _, _ = self.batch.system(self.system(ci, f))
        j = int(self.local[a])
        return self.cells[ci].members, X[:, j], Y[:, j]

    def patterns(self, models_list, f: int, theta: torch.Tensor, phi: torch.Tensor) -> torch.Tensor:
        """Embedded element patterns E[a, dir, (theta, phi)] of every antenna at
        model index f (Eqs. 5-6 over its subarray's currents); models_list[f]
        is the Model of that frequency."""
        dev = theta.device
        E = torch.empty((self.x.size, int(theta.numel()), 2), dtype=torch.complex128, device=dev)
        for ci, c in enumerate(self.cells):
            X, _, _, _ = self.batch.system(self.system(ci, f))
            xs = torch.from_numpy(self.x[c.members]).to(dev)
            ys = torch.from_numpy(self.y[c.members]).to(dev)
            Ec = embedded_patterns(models_list[f], xs, ys, X, theta, phi)
            E[torch.from_numpy(c.members[:c.n_inner]).to(dev)] = Ec
        return E


def prof_enable(on: bool) -> None:
    check(lib().harp_prof_enable(1 if on else 0), "harp_prof_enable")


PROF_CLASSES = ["fill", "getf2", "trsm_lower", "trsm_upper", "gemm_c64", "gemm_c128", "aux", "rank_update"]


GEMM_SITES = ["other", "trailing", "catch_up", "deferred_rows", "block_row", "tri_inverse", "solve_diag",
              "solve_update", "residual", "residual_update"]


def prof_read_sites() -> dict:
    """Per call site of the two GEMM classes: launches, ms, flops, bytes."""
    out = {}
    for cls, cname in ((4, "gemm_c64"), (5, "gemm_c128")):
        for i, site in enumerate(GEMM_SITES):
            n = ctypes.c_int64()
            ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            check(lib().harp_prof_read_site(cls, i, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                                            ctypes.byref(by)), "harp_prof_read_site")
            if n.value:
                out[f"{cname}.{site}"] = {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}
    return out


def prof_read() -> dict:
    out = {}
    for i, name in enumerate(PROF_CLASSES):
        n = ctypes.c_int64()
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(lib().harp_prof_read(i, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                                   ctypes.byref(by)), "harp_prof_read")
        out[name] = {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}
    return out
