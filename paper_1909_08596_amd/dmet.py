"""ctypes binding of libdmet.so (argument marshalling only).

Every function takes and returns torch tensors that live on the current HIP
device; torch provides device memory and the stream, the library does all
arithmetic.  The binding refuses to run without the compiled library: there is
no CPU fallback.  Names and arguments mirror include/dmet.h.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmet.so")

DMET_FP64, DMET_FP32_3M, DMET_BF16X3_3M, DMET_BF16X6_3M, DMET_BF16X6_I8 = 0, 1, 2, 3, 4
DMET_C128, DMET_C64 = 0, 1
PRECISIONS = {"fp64": DMET_FP64, "fp32": DMET_FP32_3M, "bf16x3": DMET_BF16X3_3M, "bf16x6": DMET_BF16X6_3M,
              "bf16x6_i8": DMET_BF16X6_I8}
STATUS = {0: "DMET_OK", 1: "DMET_E_ARG", 2: "DMET_E_HIP", 3: "DMET_E_NOCONV", 4: "DMET_E_RANK",
          5: "DMET_E_NONFINITE", 6: "DMET_E_WORKSPACE", 7: "DMET_E_UNSUPPORTED"}

# every symbol include/dmet.h declares
EXPORTS = ("dmet_last_error", "dmet_version", "dmet_build_bath_workspace", "dmet_build_bath",
           "dmet_build_bath_noalloc",
           "dmet_transform_1e", "dmet_energy_1e", "dmet_transform_eri_workspace", "dmet_transform_eri",
           "dmet_transform_eri_batched_workspace", "dmet_transform_eri_batched",
           "dmet_transform_eri_df", "dmet_transform_eri_fftdf_workspace", "dmet_transform_eri_fftdf",
           "dmet_transform_eri_impurity_workspace", "dmet_transform_eri_impurity",
           "dmet_fock_dc_workspace", "dmet_fock_dc", "dmet_energy_mf",
           "dmet_profile_enable", "dmet_profile_reset", "dmet_profile_report")
DMET_BATCH_GRAPH, DMET_BATCH_AUTOTUNE = 1, 2


class DmetError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Lattice(ctypes.Structure):
    _fields_ = [("kmesh", ctypes.c_int * 3), ("nao", ctypes.c_int), ("naux", ctypes.c_int),
                ("nspin", ctypes.c_int)]


def lattice(kmesh: Sequence[int], nao: int, naux: int = 1, nspin: int = 1) -> Lattice:
    lat = Lattice()
    for d in range(3):
        lat.kmesh[d] = int(kmesh[d])
    lat.nao, lat.naux, lat.nspin = int(nao), int(naux), int(nspin)
    return lat


class PwGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("cell", (ctypes.c_double * 3) * 3)]


def pw_grid(n: Sequence[int], cell) -> PwGrid:
    """Grid of the plane-wave entry points: n points per axis; cell the three
    lattice vectors as rows (bohr), or three edge lengths of an orthorhombic cell."""
    g = PwGrid()
    rows = list(cell)
    if len(rows) != 3:
        raise ValueError("cell: three edge lengths or three lattice vectors")
    for d in range(3):
        g.n[d] = int(n[d])
        if isinstance(rows[d], (int, float)):
            for c in range(3):
                g.cell[d][c] = float(rows[d]) if c == d else 0.0
        else:
            vec = [float(x) for x in rows[d]]
            if len(vec) != 3:
                raise ValueError("cell: each lattice vector has three components")
            for c in range(3):
                g.cell[d][c] = vec[c]
    return g


class Fragment(ctypes.Structure):
    _fields_ = [("lat", Lattice), ("neo", ctypes.c_int), ("lmunu", ctypes.c_void_p), ("dtype", ctypes.c_int),
                ("c_k", ctypes.c_void_p), ("eri", ctypes.c_void_p)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdmet.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1909_08596_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lp = ctypes.POINTER(Lattice)
    lib.dmet_last_error.restype = ctypes.c_char_p
    lib.dmet_last_error.argtypes = []
    lib.dmet_version.restype = i
    lib.dmet_build_bath_workspace.argtypes = [lp, i, i, ctypes.POINTER(sz)]
    lib.dmet_build_bath.argtypes = [lp, vp, i, vp, i, vp, d, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.dmet_build_bath_noalloc.argtypes = [lp, vp, i, vp, i, vp, d, vp, vp, vp, vp, vp, vp]
    lib.dmet_transform_1e.argtypes = [lp, i, vp, vp, vp, vp, vp]
    lib.dmet_energy_1e.argtypes = [i, i, vp, vp, vp, vp]
    lib.dmet_transform_eri_workspace.argtypes = [lp, i, i, i, ctypes.POINTER(sz)]
    lib.dmet_transform_eri.argtypes = [lp, i, vp, i, vp, i, vp, vp, vp, vp, sz, vp]
    fp = ctypes.POINTER(Fragment)
    lib.dmet_transform_eri_batched_workspace.argtypes = [i, fp, i, ctypes.POINTER(sz)]
    lib.dmet_transform_eri_batched.argtypes = [i, fp, i, ctypes.c_uint, vp, sz, vp]
    lib.dmet_transform_eri_df.argtypes = [lp, i, vp, i, vp, i, vp, vp, sz, vp]
    lib.dmet_transform_eri_impurity_workspace.argtypes = [lp, i, i, i, i, ctypes.POINTER(sz)]
    lib.dmet_transform_eri_impurity.argtypes = [lp, i, i, vp, i, vp, i, vp, vp, vp, vp, sz, vp]
    gp = ctypes.POINTER(PwGrid)
    lib.dmet_transform_eri_fftdf_workspace.argtypes = [lp, gp, i, i, i, ctypes.POINTER(sz)]
    lib.dmet_transform_eri_fftdf.argtypes = [lp, gp, i, vp, i, i, vp, vp, vp, vp, vp, sz, vp]
    lib.dmet_fock_dc_workspace.argtypes = [i, i, i, ctypes.POINTER(sz)]
    lib.dmet_fock_dc.argtypes = [i, i, i, vp, vp, vp, vp, vp, sz, vp]
    lib.dmet_energy_mf.argtypes = [i, i, vp, vp, vp, vp, vp]
    lib.dmet_profile_enable.argtypes = [i]
    lib.dmet_profile_reset.argtypes = []
    lib.dmet_profile_report.argtypes = [ctypes.c_char_p, sz]
    for name in EXPORTS:
        if name not in ("dmet_last_error", "dmet_version"):
            getattr(lib, name).restype = i
    _lib = lib
    return lib


def _check(st: int):
    if st != 0:
        raise DmetError(st, load().dmet_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _shape(t, shape, name):
    """The library receives raw pointers, so every extent is checked here:
    a tensor of the wrong shape would make the kernels read or write past it."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    want = tuple(int(x) for x in shape)
    if tuple(t.shape) != want:
        raise ValueError(f"{name} must have shape {want}, got {tuple(t.shape)}")
    return t


def _nk(kmesh) -> int:
    if len(kmesh) != 3 or any(int(x) < 1 for x in kmesh):
        raise ValueError("kmesh must be three positive integers")
    return int(kmesh[0]) * int(kmesh[1]) * int(kmesh[2])


def _dev(t: torch.Tensor, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def dmet_build_bath(kmesh, nao, dm_k: torch.Tensor, imp_idx=None, val_idx=None, sv_tol: float = 0.0,
                    c_ao_lo: Optional[torch.Tensor] = None, stream=None, return_imag: bool = False):
    """Bath SVD and embedding coefficients.  Returns (c_k, sv, neo list), and
    max |Im gamma^{R,0}| as a fourth item if return_imag; c_k has nimp + nval
    columns, those past neo[s] are zero."""
    lib = load()
    nk = _nk(kmesh)
    if dm_k.dim() != 4 or dm_k.shape[0] not in (1, 2):
        raise ValueError("dm_k must be [nspin][N_k][nao][nao] with nspin 1 or 2")
    nspin = dm_k.shape[0]
    _shape(dm_k, (nspin, nk, nao, nao), "dm_k")
    if c_ao_lo is not None:
        _shape(c_ao_lo, (nk, nao, nao), "c_ao_lo")
        _dev(c_ao_lo, torch.complex128, "c_ao_lo")
    _dev(dm_k, torch.complex128, "dm_k")
    lat = lattice(kmesh, nao, 1, nspin)
    nimp = nao if imp_idx is None else len(imp_idx)
    nval = nimp if val_idx is None else len(val_idx)
    imp_arr = None if imp_idx is None else (ctypes.c_int * nimp)(*[int(x) for x in imp_idx])
    val_arr = None if val_idx is None else (ctypes.c_int * nval)(*[int(x) for x in val_idx])
    c_k = torch.empty((nspin, nk, nao, nimp + nval), dtype=torch.complex128, device=dm_k.device)
    sv = torch.empty((nspin, nval), dtype=torch.float64, device=dm_k.device)
    nb = ctypes.c_size_t()
    _check(lib.dmet_build_bath_workspace(ctypes.byref(lat), nimp, nval, ctypes.byref(nb)))
    ws = _workspace(nb.value, dm_k.device)
    neo = (ctypes.c_int * nspin)()
    mi = ctypes.c_double(-1.0)
    _check(lib.dmet_build_bath(ctypes.byref(lat), _ptr(dm_k), nimp, imp_arr, nval, val_arr, float(sv_tol),
                               _ptr(c_ao_lo), _ptr(c_k), _ptr(sv), neo, ctypes.byref(mi), _ptr(ws), ws.numel(),
                               _stream(stream)))
    if return_imag:
        return c_k, sv, [int(x) for x in neo], mi.value
    return c_k, sv, [int(x) for x in neo]


def dmet_build_bath_noalloc(kmesh, nao, dm_k: torch.Tensor, imp_idx=None, val_idx=None, sv_tol: float = 0.0,
                            c_ao_lo: Optional[torch.Tensor] = None, c_k: Optional[torch.Tensor] = None,
                            sv: Optional[torch.Tensor] = None, stream=None):
    """dmet_build_bath on the library's own per-GPU scratch (no workspace);
    c_k and sv may be preallocated by the caller.  Returns (c_k, sv, neo list,
    max |Im gamma^{R,0}|)."""
    lib = load()
    nk = _nk(kmesh)
    if dm_k.dim() != 4 or dm_k.shape[0] not in (1, 2):
        raise ValueError("dm_k must be [nspin][N_k][nao][nao] with nspin 1 or 2")
    nspin = dm_k.shape[0]
    _shape(dm_k, (nspin, nk, nao, nao), "dm_k")
    nimp = nao if imp_idx is None else len(imp_idx)
    nval = nimp if val_idx is None else len(val_idx)
    if c_ao_lo is not None:
        _shape(c_ao_lo, (nk, nao, nao), "c_ao_lo")
        _dev(c_ao_lo, torch.complex128, "c_ao_lo")
    if c_k is None:
        c_k = torch.empty((nspin, nk, nao, nimp + nval), dtype=torch.complex128, device=dm_k.device)
    if sv is None:
        sv = torch.empty((nspin, nval), dtype=torch.float64, device=dm_k.device)
    _shape(c_k, (nspin, nk, nao, nimp + nval), "c_k")
    _shape(sv, (nspin, nval), "sv")
    _dev(dm_k, torch.complex128, "dm_k")
    _dev(c_k, torch.complex128, "c_k")
    _dev(sv, torch.float64, "sv")
    lat = lattice(kmesh, nao, 1, nspin)
    imp_arr = None if imp_idx is None else (ctypes.c_int * nimp)(*[int(x) for x in imp_idx])
    val_arr = None if val_idx is None else (ctypes.c_int * nval)(*[int(x) for x in val_idx])
    neo = (ctypes.c_int * nspin)()
    mi = ctypes.c_double(-1.0)
    _check(lib.dmet_build_bath_noalloc(ctypes.byref(lat), _ptr(dm_k), nimp, imp_arr, nval, val_arr, float(sv_tol),
                                       _ptr(c_ao_lo), _ptr(c_k), _ptr(sv), neo, ctypes.byref(mi), _stream(stream)))
    return c_k, sv, [int(x) for x in neo], mi.value


def dmet_transform_1e(kmesh, nao, c_k: torch.Tensor, op_k: torch.Tensor, want_imag: bool = False, stream=None):
    """X^{0,EO} = 1/N_k sum_k C^k^H X^k C^k.  Returns (op_eo, max |Im| as a
    float, or None); asking for max |Im| synchronises the stream."""
    lib = load()
    nk = _nk(kmesh)
    if c_k.dim() != 4 or c_k.shape[0] not in (1, 2):
        raise ValueError("c_k must be [nspin][N_k][nao][neo] with nspin 1 or 2")
    nspin, neo = c_k.shape[0], c_k.shape[3]
    _shape(c_k, (nspin, nk, nao, neo), "c_k")
    _shape(op_k, (nspin, nk, nao, nao), "op_k")
    _dev(c_k, torch.complex128, "c_k")
    _dev(op_k, torch.complex128, "op_k")
    lat = lattice(kmesh, nao, 1, nspin)
    out = torch.empty((nspin, neo, neo), dtype=torch.float64, device=c_k.device)
    mi = ctypes.c_double(-1.0)
    _check(lib.dmet_transform_1e(ctypes.byref(lat), neo, _ptr(c_k), _ptr(op_k), _ptr(out),
                                 ctypes.byref(mi) if want_imag else None, _stream(stream)))
    return out, (mi.value if want_imag else None)


def dmet_energy_1e(h_eo: torch.Tensor, dm_eo: torch.Tensor, stream=None) -> torch.Tensor:
    lib = load()
    if h_eo.dim() != 3 or h_eo.shape[0] not in (1, 2) or h_eo.shape[1] != h_eo.shape[2]:
        raise ValueError("h_eo must be [nspin][neo][neo] with nspin 1 or 2")
    _shape(dm_eo, h_eo.shape, "dm_eo")
    _dev(h_eo, torch.float64, "h_eo")
    _dev(dm_eo, torch.float64, "dm_eo")
    e1 = torch.empty(1, dtype=torch.float64, device=h_eo.device)
    _check(lib.dmet_energy_1e(h_eo.shape[0], h_eo.shape[1], _ptr(h_eo), _ptr(dm_eo), _ptr(e1), _stream(stream)))
    return e1


def dmet_transform_eri_workspace(kmesh, nao, naux, nspin, neo, precision="fp64", dtype=torch.complex128) -> int:
    lib = load()
    lat = lattice(kmesh, nao, naux, nspin)
    nb = ctypes.c_size_t()
    dt = DMET_C128 if dtype == torch.complex128 else DMET_C64
    _check(lib.dmet_transform_eri_workspace(ctypes.byref(lat), int(neo), PRECISIONS[precision], dt,
                                            ctypes.byref(nb)))
    return nb.value


def _eri_inputs(kmesh, nao, naux, lmunu, c_k, name="lmunu"):
    """Shape, dtype and device checks of the 3-index tensor and C^k; returns (nspin, neo)."""
    nk = _nk(kmesh)
    if not isinstance(lmunu, torch.Tensor) or lmunu.dtype not in (torch.complex128, torch.complex64):
        raise ValueError(f"{name} must be complex128 or complex64")
    if not isinstance(c_k, torch.Tensor) or c_k.dim() != 4 or c_k.shape[0] not in (1, 2):
        raise ValueError("c_k must be [nspin][N_k][nao][neo] with nspin 1 or 2")
    nspin, neo = c_k.shape[0], c_k.shape[3]
    _shape(lmunu, (nk, nk, naux, nao, nao), name)
    _shape(c_k, (nspin, nk, nao, neo), "c_k")
    _dev(lmunu, lmunu.dtype, name)
    _dev(c_k, torch.complex128, "c_k")
    return nspin, neo


def _eri_outputs(out, nspin, npair):
    """Caller-supplied output tensors must hold the packed blocks the call writes."""
    s8 = npair * (npair + 1) // 2
    if "aa" not in out:
        raise ValueError("out needs an 'aa' tensor")
    want = {"aa": (s8,), "bb": (s8,), "ab": (npair, npair)}
    for key, t in out.items():
        if key not in want:
            raise ValueError(f"unknown output block {key!r}")
        if nspin == 1 and key != "aa":
            raise ValueError("one spin writes only the 'aa' block")
        if t.numel() != math.prod(want[key]):
            raise ValueError(f"out[{key!r}] must hold {want[key]} float64 values, got {tuple(t.shape)}")
    if nspin == 2 and "bb" not in out:
        raise ValueError("two spins need a 'bb' output")
    for key, t in out.items():
        _dev(t, torch.float64, f"out[{key!r}]")


def _workspace_ok(ws, need):
    _dev(ws, torch.uint8, "workspace")
    if ws.numel() < need:
        raise ValueError(f"workspace holds {ws.numel()} bytes, the call needs {need}")


def dmet_transform_eri(kmesh, nao, naux, lmunu: torch.Tensor, c_k: torch.Tensor, precision: str = "fp64",
                       eri_ab: bool = True, workspace: Optional[torch.Tensor] = None, out=None, stream=None):
    """Packed embedding ERIs by Alg. 1.  Returns dict with 'aa' (s8), and for
    two spins 'bb' (s8) and 'ab' (s4, if requested)."""
    lib = load()
    nspin, neo = _eri_inputs(kmesh, nao, naux, lmunu, c_k)
    lat = lattice(kmesh, nao, naux, nspin)
    dt = DMET_C128 if lmunu.dtype == torch.complex128 else DMET_C64
    npair = neo * (neo + 1) // 2
    dev = c_k.device
    if out is None:
        out = {"aa": torch.empty(npair * (npair + 1) // 2, dtype=torch.float64, device=dev)}
        if nspin == 2:
            out["bb"] = torch.empty_like(out["aa"])
            if eri_ab:
                out["ab"] = torch.empty((npair, npair), dtype=torch.float64, device=dev)
    _eri_outputs(out, nspin, npair)
    need = dmet_transform_eri_workspace(kmesh, nao, naux, nspin, neo, precision, lmunu.dtype)
    if workspace is None:
        workspace = _workspace(need, dev)
    _workspace_ok(workspace, need)
    _check(lib.dmet_transform_eri(ctypes.byref(lat), neo, _ptr(lmunu), dt, _ptr(c_k), PRECISIONS[precision],
                                  _ptr(out["aa"]), _ptr(out.get("bb")), _ptr(out.get("ab")), _ptr(workspace),
                                  workspace.numel(), _stream(stream)))
    return out


def dmet_transform_eri_impurity(kmesh, nao, naux, lmunu: torch.Tensor, c_k: torch.Tensor, nimp: int,
                                precision: str = "fp64", eri_ab: bool = True, stream=None):
    """ERIs of the non-interacting-bath formalism (Sec. 2.1): two-particle
    terms on the impurity orbitals only, i.e. Alg. 1 on the first nimp columns
    of C^k (the impurity block of Eq. ``C loemb k``).  Same return value as
    dmet_transform_eri with neo = nimp."""
    lib = load()
    nspin, neo = _eri_inputs(kmesh, nao, naux, lmunu, c_k)
    if not 1 <= nimp <= neo:
        raise ValueError("need 1 <= nimp <= neo")
    lat = lattice(kmesh, nao, naux, nspin)
    dt = DMET_C128 if lmunu.dtype == torch.complex128 else DMET_C64
    npair = nimp * (nimp + 1) // 2
    dev = c_k.device
    out = {"aa": torch.empty(npair * (npair + 1) // 2, dtype=torch.float64, device=dev)}
    if nspin == 2:
        out["bb"] = torch.empty_like(out["aa"])
        if eri_ab:
            out["ab"] = torch.empty((npair, npair), dtype=torch.float64, device=dev)
    nb = ctypes.c_size_t()
    _check(lib.dmet_transform_eri_impurity_workspace(ctypes.byref(lat), neo, int(nimp), PRECISIONS[precision], dt,
                                                     ctypes.byref(nb)))
    ws = _workspace(nb.value, dev)
    _check(lib.dmet_transform_eri_impurity(ctypes.byref(lat), neo, int(nimp), _ptr(lmunu), dt, _ptr(c_k),
                                           PRECISIONS[precision], _ptr(out["aa"]), _ptr(out.get("bb")),
                                           _ptr(out.get("ab")), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def dmet_transform_eri_fftdf(kmesh, nao, grid_n, cell, rho: torch.Tensor, c_k: torch.Tensor, eri_ab: bool = True,
                             workspace: Optional[torch.Tensor] = None, stream=None, precision: str = "fp64"):
    """Plane-wave (FFTDF) embedding ERIs (App. B, Alg. 2).  rho is the AO pair
    density on the cell grid [q][k][r][mu][nu] = (r|mu k, nu k-q), grid_n the
    grid points per axis and cell the three lattice vectors as rows (bohr) or
    the three edge lengths of an orthorhombic cell; precision "fp64", "bf16x6"
    or "bf16x3" (the transform and contraction in that form, the grid DFT in
    FP64).  Same return value as dmet_transform_eri."""
    lib = load()
    nr = int(grid_n[0]) * int(grid_n[1]) * int(grid_n[2])
    nspin, neo = _eri_inputs(kmesh, nao, nr, rho, c_k, "rho")
    lat = lattice(kmesh, nao, nr, nspin)
    grid = pw_grid(grid_n, cell)
    dt = DMET_C128 if rho.dtype == torch.complex128 else DMET_C64
    npair = neo * (neo + 1) // 2
    dev = c_k.device
    out = {"aa": torch.empty(npair * (npair + 1) // 2, dtype=torch.float64, device=dev)}
    if nspin == 2:
        out["bb"] = torch.empty_like(out["aa"])
        if eri_ab:
            out["ab"] = torch.empty((npair, npair), dtype=torch.float64, device=dev)
    nb = ctypes.c_size_t()
    prec = PRECISIONS[precision]
    _check(lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(grid), neo, dt, prec,
                                                  ctypes.byref(nb)))
    if workspace is None:
        workspace = _workspace(nb.value, dev)
    _workspace_ok(workspace, nb.value)
    _check(lib.dmet_transform_eri_fftdf(ctypes.byref(lat), ctypes.byref(grid), neo, _ptr(rho), dt, prec, _ptr(c_k),
                                        _ptr(out["aa"]), _ptr(out.get("bb")), _ptr(out.get("ab")), _ptr(workspace),
                                        workspace.numel(), _stream(stream)))
    return out


def dmet_transform_eri_df(kmesh, nao, naux, lmunu: torch.Tensor, c_k: torch.Tensor, precision: str = "fp64",
                          workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Density-fitting factors z [nspin][N_k*naux][npair] (float64) with
    (ij|kl)_st = sum_P z_s[P][ij] z_t[P][kl] (the contraction of Alg. 1 skipped)."""
    lib = load()
    nspin, neo = _eri_inputs(kmesh, nao, naux, lmunu, c_k)
    nk = _nk(kmesh)
    lat = lattice(kmesh, nao, naux, nspin)
    dt = DMET_C128 if lmunu.dtype == torch.complex128 else DMET_C64
    npair = neo * (neo + 1) // 2
    z = torch.empty((nspin, nk * naux, npair), dtype=torch.float64, device=c_k.device)
    need = dmet_transform_eri_workspace(kmesh, nao, naux, nspin, neo, precision, lmunu.dtype)
    if workspace is None:
        workspace = _workspace(need, c_k.device)
    _workspace_ok(workspace, need)
    _check(lib.dmet_transform_eri_df(ctypes.byref(lat), neo, _ptr(lmunu), dt, _ptr(c_k), PRECISIONS[precision],
                                     _ptr(z), _ptr(workspace), workspace.numel(), _stream(stream)))
    return z


def dmet_fock_dc(z: torch.Tensor, f_eo: torch.Tensor, dm_eo: torch.Tensor, stream=None) -> torch.Tensor:
    """F~ of Eq. "fock double counting" from the DF factors z, F^EO and the
    per-spin embedding density (all float64 device tensors)."""
    lib = load()
    if f_eo.dim() != 3 or f_eo.shape[0] not in (1, 2) or f_eo.shape[1] != f_eo.shape[2]:
        raise ValueError("f_eo must be [nspin][neo][neo] with nspin 1 or 2")
    nspin, neo = f_eo.shape[0], f_eo.shape[1]
    if z.dim() != 3:
        raise ValueError("z must be [nspin][nrows][npair]")
    nrows = z.shape[1]
    _shape(z, (nspin, nrows, neo * (neo + 1) // 2), "z")
    _shape(dm_eo, f_eo.shape, "dm_eo")
    _dev(z, torch.float64, "z")
    _dev(f_eo, torch.float64, "f_eo")
    _dev(dm_eo, torch.float64, "dm_eo")
    nb = ctypes.c_size_t()
    _check(lib.dmet_fock_dc_workspace(nspin, neo, nrows, ctypes.byref(nb)))
    ws = _workspace(nb.value, f_eo.device)
    out = torch.empty_like(f_eo)
    _check(lib.dmet_fock_dc(nspin, neo, nrows, _ptr(z), _ptr(f_eo), _ptr(dm_eo), _ptr(out), _ptr(ws), ws.numel(),
                            _stream(stream)))
    return out


def dmet_energy_mf(f_tilde: torch.Tensor, f_eo: torch.Tensor, dm_eo: torch.Tensor, stream=None) -> torch.Tensor:
    """Mean-field (Hartree-Fock form) energy of the embedding Hamiltonian with
    one-body part F~ (float64 device tensors [nspin][neo][neo]); device [1]."""
    lib = load()
    if f_eo.dim() != 3 or f_eo.shape[0] not in (1, 2) or f_eo.shape[1] != f_eo.shape[2]:
        raise ValueError("f_eo must be [nspin][neo][neo] with nspin 1 or 2")
    _shape(f_tilde, f_eo.shape, "f_tilde")
    _shape(dm_eo, f_eo.shape, "dm_eo")
    _dev(f_tilde, torch.float64, "f_tilde")
    _dev(f_eo, torch.float64, "f_eo")
    _dev(dm_eo, torch.float64, "dm_eo")
    e = torch.empty(1, dtype=torch.float64, device=f_eo.device)
    _check(lib.dmet_energy_mf(f_eo.shape[0], f_eo.shape[1], _ptr(f_tilde), _ptr(f_eo), _ptr(dm_eo), _ptr(e),
                              _stream(stream)))
    return e


def _fragments(frags, precision):
    for n, f in enumerate(frags):
        nk = _nk(f["kmesh"])
        ck = f["c_k"]
        if not isinstance(ck, torch.Tensor) or ck.dim() != 3:
            raise ValueError(f"fragment {n}: c_k must be [N_k][nao][neo]")
        neo = ck.shape[-1]
        npair = neo * (neo + 1) // 2
        _shape(ck, (nk, f["nao"], neo), f"fragment {n}: c_k")
        lm = f["lmunu"]
        if not isinstance(lm, torch.Tensor) or lm.dtype not in (torch.complex128, torch.complex64):
            raise ValueError(f"fragment {n}: lmunu must be complex128 or complex64")
        _shape(lm, (nk, nk, f["naux"], f["nao"], f["nao"]), f"fragment {n}: lmunu")
        if "eri" not in f:
            f["eri"] = torch.empty(npair * (npair + 1) // 2, dtype=torch.float64, device=ck.device)
        if f["eri"].numel() != npair * (npair + 1) // 2:
            raise ValueError(f"fragment {n}: eri must hold {npair * (npair + 1) // 2} float64 values")
        _dev(f["eri"], torch.float64, f"fragment {n}: eri")
    arr = (Fragment * len(frags))()
    for n, f in enumerate(frags):
        lm, ck = f["lmunu"], f["c_k"]
        _dev(lm, lm.dtype, "lmunu")
        _dev(ck, torch.complex128, "c_k")
        neo = ck.shape[-1]
        arr[n].lat = lattice(f["kmesh"], f["nao"], f["naux"], 1)
        arr[n].neo = neo
        arr[n].lmunu = lm.data_ptr()
        arr[n].dtype = DMET_C128 if lm.dtype == torch.complex128 else DMET_C64
        arr[n].c_k = ck.data_ptr()
        arr[n].eri = f["eri"].data_ptr()
    return arr


def dmet_transform_eri_batched_workspace(frags, precision="bf16x6") -> int:
    arr = _fragments(frags, precision)
    nb = ctypes.c_size_t()
    _check(load().dmet_transform_eri_batched_workspace(len(frags), arr, PRECISIONS[precision], ctypes.byref(nb)))
    return nb.value


def dmet_transform_eri_batched(frags, precision="bf16x6", graph=False, autotune=False,
                               workspace: Optional[torch.Tensor] = None, stream=None):
    """Packed s8 ERIs of many fragments in one submission.  `frags` is a list of
    dicts with kmesh, nao, naux, lmunu, c_k ([N_k][nao][neo] complex128) and an
    optional preallocated 'eri'; returns the list of output tensors."""
    arr = _fragments(frags, precision)
    nb = ctypes.c_size_t()
    _check(load().dmet_transform_eri_batched_workspace(len(frags), arr, PRECISIONS[precision], ctypes.byref(nb)))
    if workspace is None:
        workspace = _workspace(nb.value, frags[0]["c_k"].device)
    _workspace_ok(workspace, nb.value)
    flags = (DMET_BATCH_GRAPH if graph else 0) | (DMET_BATCH_AUTOTUNE if autotune else 0)
    _check(load().dmet_transform_eri_batched(len(frags), arr, PRECISIONS[precision], flags, _ptr(workspace),
                                             workspace.numel(), _stream(stream)))
    return [f["eri"] for f in frags]


def dmet_profile_enable(on: bool = True):
    _check(load().dmet_profile_enable(1 if on else 0))


def dmet_profile_reset():
    _check(load().dmet_profile_reset())


def dmet_profile_report() -> dict:
    """{kernel name: (launches, total ms)} since the last reset (waits for the events)."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load().dmet_profile_report(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.split()
        out[name] = (int(n), float(ms))
    return out
