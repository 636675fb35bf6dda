"""ctypes binding of libmderi (see include/mderi.h for the contract)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmderi.so")

_lib = None

MDERI_LMAX = 8
MDERI_KMAX = 16


class MderiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libmderi status {status}: {msg}")
        self.status = status


def lib_path() -> str:
    return _LIB_PATH


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("schwarz_tau", ctypes.c_double), ("flags", ctypes.c_int),
                ("split_slices", ctypes.c_int), ("tile_variant", ctypes.c_int), ("deterministic", ctypes.c_int)]


FLAG_GRAPH = 1
FLAG_AUTOTUNE = 2
FLAG_SYMMETRIC = 4
FP64 = 0
SPLIT_BF16 = 1
SPLIT_FP32 = 2  # declared by the ABI, not built (MDERI_EUNSUPPORTED)
EXCHANGE = 0
COULOMB = 1


_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)


def load_library():
    """Loads libmderi.so (built by paper_2405_01834_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise MderiError(-3, f"{_LIB_PATH} is not built (run paper_2405_01834_amd/build.py)")
    L = ctypes.CDLL(_LIB_PATH)
    L.mderi_create.argtypes = [ctypes.c_int, ctypes.POINTER(_vp)]
    L.mderi_create.restype = ctypes.c_int
    L.mderi_destroy.argtypes = [_vp]
    L.mderi_destroy.restype = None
    L.mderi_last_error.argtypes = []
    L.mderi_last_error.restype = ctypes.c_char_p
    L.mderi_basis_upload.argtypes = [_vp, ctypes.c_int, _ip, _ip, _dp, _dp, _dp, _ip, ctypes.c_int, ctypes.POINTER(_vp)]
    L.mderi_basis_upload.restype = ctypes.c_int
    L.mderi_basis_free.argtypes = [_vp]
    L.mderi_basis_free.restype = None
    L.mderi_basis_nshell.argtypes = [_vp]
    L.mderi_basis_nshell.restype = ctypes.c_int
    L.mderi_basis_nao.argtypes = [_vp]
    L.mderi_basis_nao.restype = ctypes.c_int
    L.mderi_eri4.argtypes = [_vp, _vp, ctypes.c_int, _ip, ctypes.c_int, _ip, _vp, ctypes.c_size_t,
                             ctypes.POINTER(Opts), _vp]
    L.mderi_eri4.restype = ctypes.c_int
    L.mderi_eri4_tile_variants.argtypes = [_vp, _vp, ctypes.c_int, _ip, ctypes.c_int, _ip, ctypes.POINTER(ctypes.c_int)]
    L.mderi_eri4_tile_variants.restype = ctypes.c_int
    L.mderi_eri4_noalloc.argtypes = [_vp, _vp, ctypes.c_int, _ip, ctypes.c_int, _ip, _vp, ctypes.c_size_t,
                                     ctypes.POINTER(Opts), _vp]
    L.mderi_eri4_noalloc.restype = ctypes.c_int
    L.mderi_eri3.argtypes = [_vp, _vp, _vp, ctypes.c_int, _ip, ctypes.c_int, _ip, _vp, ctypes.c_size_t,
                             ctypes.POINTER(Opts), _vp]
    L.mderi_eri3.restype = ctypes.c_int
    L.mderi_eri2.argtypes = [_vp, _vp, ctypes.c_int, _ip, ctypes.c_int, _ip, _vp, ctypes.c_size_t,
                             ctypes.POINTER(Opts), _vp]
    L.mderi_eri2.restype = ctypes.c_int
    L.mderi_dfj.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(Opts), _vp]
    L.mderi_dfj.restype = ctypes.c_int
    L.mderi_dfk.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(Opts), _vp]
    L.mderi_dfk.restype = ctypes.c_int
    L.mderi_kbuild.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(Opts), _vp]
    L.mderi_kbuild.restype = ctypes.c_int
    L.mderi_eri3_batch.argtypes = [_vp, _vp, _vp, ctypes.c_int, _ip, ctypes.c_int, _ip, _vp, ctypes.c_size_t,
                                   ctypes.POINTER(Opts), _vp]
    L.mderi_eri3_batch.restype = ctypes.c_int
    L.mderi_kernel_timing.argtypes = [_vp, ctypes.c_int]
    L.mderi_kernel_timing.restype = ctypes.c_int
    L.mderi_progress.argtypes = [_vp, ctypes.c_int]
    L.mderi_progress.restype = ctypes.c_int
    L.mderi_set_workspace_limit.argtypes = [_vp, ctypes.c_size_t]
    L.mderi_set_workspace_limit.restype = ctypes.c_int
    for name in ("mderi_tune_save", "mderi_tune_load"):
        getattr(L, name).argtypes = [_vp, ctypes.c_char_p]
        getattr(L, name).restype = ctypes.c_int
    L.mderi_kernel_times.argtypes = [_vp, _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.mderi_kernel_times.restype = ctypes.c_int
    L.mderi_jkbuild.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.POINTER(Opts), _vp]
    L.mderi_jkbuild.restype = ctypes.c_int
    L.mderi_kbuild_grad.argtypes = [_vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_double, _vp, ctypes.c_int,
                                    ctypes.c_int, ctypes.POINTER(Opts), _vp]
    L.mderi_kbuild_grad.restype = ctypes.c_int
    L.mderi_basis_set_centers.argtypes = [_vp, _vp, _vp]
    L.mderi_basis_set_centers.restype = ctypes.c_int
    L.mderi_schwarz.argtypes = [_vp, _vp, ctypes.c_int, _ip, _vp, _vp]
    L.mderi_schwarz.restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise MderiError(st, load_library().mderi_last_error().decode())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def nsph(l):
    return 2 * l + 1


class Context:
    """Owns a libmderi context on one HIP device."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise MderiError(-4, "no GPU visible to torch; libmderi has no CPU path")
        self.device = device
        torch.cuda.set_device(device)
        L = load_library()
        h = _vp()
        _check(L.mderi_create(device, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().mderi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def basis(self, l, nprim, exps, coefs, centers, atom=None, normalize=1) -> "Basis":
        return Basis(self, l, nprim, exps, coefs, centers, atom, normalize)

    def eri4_tile_variants(self, basis: "Basis", bra, ket) -> int:
        """Number of work splits the fused kernel supports for this class batch."""
        bra = np.ascontiguousarray(np.asarray(bra, dtype=np.int32).reshape(-1, 2))
        ket = np.ascontiguousarray(np.asarray(ket, dtype=np.int32).reshape(-1, 2))
        n = ctypes.c_int(0)
        _check(load_library().mderi_eri4_tile_variants(self._h, basis._h, len(bra), bra.ctypes.data_as(_ip), len(ket),
                                                       ket.ctypes.data_as(_ip), ctypes.byref(n)))
        return n.value

    def eri4(self, basis: "Basis", bra, ket, out=None, stream=None, flags=0, precision=0, slices=0, tile_variant=0):
        """Class batch (ab|cd) -> torch float64 tensor V[ij, ab, cd, kl] (shape
        (nbra, Nab, Ncd, nket), a Fortran-order view of the flat output)."""
        import torch
        bra = np.ascontiguousarray(np.asarray(bra, dtype=np.int32).reshape(-1, 2))
        ket = np.ascontiguousarray(np.asarray(ket, dtype=np.int32).reshape(-1, 2))
        nab, ncd = basis.pair_dim(bra), basis.pair_dim(ket)
        if nab is None or ncd is None:  # let the library report the bad index
            _check(load_library().mderi_eri4(self._h, basis._h, len(bra), bra.ctypes.data_as(_ip), len(ket),
                                             ket.ctypes.data_as(_ip), None, 0, None, _stream_handle(stream)))
        n = len(bra) * nab * ncd * len(ket)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=f"cuda:{self.device}")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        opts = Opts(int(precision), 1e-12, int(flags), int(slices), int(tile_variant))
        _check(load_library().mderi_eri4(self._h, basis._h, len(bra), bra.ctypes.data_as(_ip), len(ket),
                                         ket.ctypes.data_as(_ip), _vp(out.data_ptr()), out.numel(),
                                         ctypes.byref(opts), _stream_handle(stream)))
        return out[:n].view(len(ket), ncd, nab, len(bra)).permute(3, 2, 1, 0)

    def eri4_noalloc(self, basis: "Basis", bra, ket, out, stream=None):
        """mderi_eri4_noalloc into the caller's float64 device tensor `out` (no
        allocation inside the call) -> the same V[ij, ab, cd, kl] view as eri4."""
        import torch
        bra = np.ascontiguousarray(np.asarray(bra, dtype=np.int32).reshape(-1, 2))
        ket = np.ascontiguousarray(np.asarray(ket, dtype=np.int32).reshape(-1, 2))
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        _check(load_library().mderi_eri4_noalloc(self._h, basis._h, len(bra), bra.ctypes.data_as(_ip), len(ket),
                                                 ket.ctypes.data_as(_ip), _vp(out.data_ptr()), out.numel(), None,
                                                 _stream_handle(stream)))
        nab, ncd = basis.pair_dim(bra), basis.pair_dim(ket)
        n = len(bra) * nab * ncd * len(ket)
        return out[:n].view(len(ket), ncd, nab, len(bra)).permute(3, 2, 1, 0)

    def eri3(self, basis: "Basis", aux: "Basis", pairs, auxidx, out=None, stream=None):
        """Class batch (ab|P) -> torch float64 tensor V[ij, ab, mP, k] (shape
        (npair, Nab, NP, naux), a Fortran-order view of the flat output)."""
        import torch
        pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        auxidx = np.ascontiguousarray(np.asarray(auxidx, dtype=np.int32).reshape(-1))
        nab = basis.pair_dim(pairs)
        ok_aux = len(auxidx) > 0 and auxidx.min() >= 0 and auxidx.max() < aux.nshell
        if nab is None or not ok_aux:
            _check(load_library().mderi_eri3(self._h, basis._h, aux._h, len(pairs), pairs.ctypes.data_as(_ip),
                                             len(auxidx), auxidx.ctypes.data_as(_ip), None, 0, None,
                                             _stream_handle(stream)))
        npp = nsph(int(aux.l[auxidx[0]]))
        n = len(pairs) * nab * npp * len(auxidx)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=f"cuda:{self.device}")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        _check(load_library().mderi_eri3(self._h, basis._h, aux._h, len(pairs), pairs.ctypes.data_as(_ip),
                                         len(auxidx), auxidx.ctypes.data_as(_ip), _vp(out.data_ptr()), out.numel(),
                                         None, _stream_handle(stream)))
        return out[:n].view(len(auxidx), npp, nab, len(pairs)).permute(3, 2, 1, 0)

    def eri2(self, basis: "Basis", shells_a, shells_c, flags=0, out=None, stream=None):
        """Class batch of the 2-centre metric (a|c) -> torch float64 tensor
        V[i, ma, mc, k] (shape (na, N(l_a), N(l_c), nc), a Fortran-order view of
        the flat output).  flags: FLAG_AUTOTUNE."""
        import torch
        sa = np.ascontiguousarray(np.asarray(shells_a, dtype=np.int32).reshape(-1))
        sc = np.ascontiguousarray(np.asarray(shells_c, dtype=np.int32).reshape(-1))
        ok = (len(sa) > 0 and len(sc) > 0 and min(sa.min(), sc.min()) >= 0 and
              max(sa.max(), sc.max()) < basis.nshell)
        opts = Opts(0, 0.0, int(flags))
        if not ok:
            _check(load_library().mderi_eri2(self._h, basis._h, len(sa), sa.ctypes.data_as(_ip), len(sc),
                                             sc.ctypes.data_as(_ip), None, 0, ctypes.byref(opts),
                                             _stream_handle(stream)))
        na_, nc_ = nsph(int(basis.l[sa[0]])), nsph(int(basis.l[sc[0]]))
        n = len(sa) * na_ * nc_ * len(sc)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=f"cuda:{self.device}")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        _check(load_library().mderi_eri2(self._h, basis._h, len(sa), sa.ctypes.data_as(_ip), len(sc),
                                         sc.ctypes.data_as(_ip), _vp(out.data_ptr()), out.numel(), ctypes.byref(opts),
                                         _stream_handle(stream)))
        return out[:n].view(len(sc), nc_, na_, len(sa)).permute(3, 2, 1, 0)

    def dfj(self, basis: "Basis", aux: "Basis", D, out=None, stream=None):
        """Density-fitted Coulomb matrix J_ab = sum_P (ab|P) [M^-1 gamma]_P with
        gamma_Q = sum_cd (Q|cd) D_cd and the metric M = (P|Q) of `aux`; D torch
        float64 [nao, nao] on the device, symmetric -> J (same shape)."""
        import torch
        nao = basis.nao()
        assert D.dtype == torch.float64 and D.is_cuda and D.shape == (nao, nao)
        D = D.contiguous()
        if out is None:
            out = torch.empty((nao, nao), dtype=torch.float64, device=D.device)
        opts = Opts(0, 0.0)
        _check(load_library().mderi_dfj(self._h, basis._h, aux._h, _vp(D.data_ptr()), _vp(out.data_ptr()), nao,
                                        ctypes.byref(opts), _stream_handle(stream)))
        return out

    def dfk(self, basis: "Basis", aux: "Basis", D, out=None, stream=None):
        """Density-fitted exchange matrix K_ac = sum_bd sum_PQ (ab|P) [M^-1]_PQ (Q|cd)
        D_bd with the metric M = (P|Q) of `aux`; D torch float64 [nao, nao] on the
        device, symmetric -> K (same shape)."""
        import torch
        nao = basis.nao()
        assert D.dtype == torch.float64 and D.is_cuda and D.shape == (nao, nao)
        D = D.contiguous()
        if out is None:
            out = torch.empty((nao, nao), dtype=torch.float64, device=D.device)
        opts = Opts(0, 0.0)
        _check(load_library().mderi_dfk(self._h, basis._h, aux._h, _vp(D.data_ptr()), _vp(out.data_ptr()), nao,
                                        ctypes.byref(opts), _stream_handle(stream)))
        return out

    def eri3_batch(self, basis: "Basis", aux: "Basis", pairs, auxidx, flags=0, out=None, stream=None):
        """(ab|P) over pairs and auxiliary shells of any classes in one task-list
        call -> torch float64 matrix [sum_i N_ab(i), sum_k N(l_k)] (a column-major
        view): row block i = pair i, column block k = aux shell k, both in list
        order.  flags: FLAG_GRAPH, FLAG_AUTOTUNE."""
        import torch
        pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        auxidx = np.ascontiguousarray(np.asarray(auxidx, dtype=np.int32).reshape(-1))
        ok = (len(pairs) > 0 and len(auxidx) > 0 and pairs.min() >= 0 and pairs.max() < basis.nshell and
              auxidx.min() >= 0 and auxidx.max() < aux.nshell)
        opts = Opts(0, 1e-12, int(flags))
        if not ok:
            _check(load_library().mderi_eri3_batch(self._h, basis._h, aux._h, len(pairs), pairs.ctypes.data_as(_ip),
                                                   len(auxidx), auxidx.ctypes.data_as(_ip), None, 0,
                                                   ctypes.byref(opts), _stream_handle(stream)))
        nrow = int(sum(nsph(int(basis.l[a])) * nsph(int(basis.l[b])) for a, b in pairs))
        ncol = int(sum(nsph(int(aux.l[k])) for k in auxidx))
        if out is None:
            out = torch.empty(nrow * ncol, dtype=torch.float64, device=f"cuda:{self.device}")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        _check(load_library().mderi_eri3_batch(self._h, basis._h, aux._h, len(pairs), pairs.ctypes.data_as(_ip),
                                               len(auxidx), auxidx.ctypes.data_as(_ip), _vp(out.data_ptr()),
                                               out.numel(), ctypes.byref(opts), _stream_handle(stream)))
        return out[:nrow * ncol].view(ncol, nrow).t()

    def jkbuild(self, basis: "Basis", D, want_j=True, want_k=True, tau=1e-12, energies=False, stream=None,
                deterministic=False):
        """Coulomb J_ab = sum_cd (ab|cd) D_cd and exchange K_ac = sum_bd (ab|cd) D_bd
        of a symmetric density D (torch float64 [nao, nao] on the device) ->
        (J or None, K or None[, energies = float64 tensor [tr(DJ), tr(DK)]]).
        deterministic: fixed-point integer accumulation, the same bits on every run."""
        import torch
        nao = basis.nao()
        assert D.dtype == torch.float64 and D.is_cuda and D.shape == (nao, nao)
        D = D.contiguous()
        J = torch.empty((nao, nao), dtype=torch.float64, device=D.device) if want_j else None
        K = torch.empty((nao, nao), dtype=torch.float64, device=D.device) if want_k else None
        E = torch.empty(2, dtype=torch.float64, device=D.device) if energies else None
        opts = Opts(0, float(tau), 0, 0, 0, int(bool(deterministic)))
        ptr = lambda t: None if t is None else _vp(t.data_ptr())  # noqa: E731
        _check(load_library().mderi_jkbuild(self._h, basis._h, _vp(D.data_ptr()), ptr(J), ptr(K), nao, ptr(E),
                                            ctypes.byref(opts), _stream_handle(stream)))
        return (J, K, E) if energies else (J, K)

    def kbuild(self, basis: "Basis", D, tau=1e-12, out=None, stream=None, deterministic=False):
        """Exchange matrix K_ac = sum_bd (ab|cd) D_bd for a symmetric density D
        (torch float64 [nao, nao] on the device) -> K (same shape).
        deterministic: fixed-point integer accumulation, the same bits on every run."""
        import torch
        nao = basis.nao()
        assert D.dtype == torch.float64 and D.is_cuda and D.shape == (nao, nao)
        D = D.contiguous()
        if out is None:
            out = torch.empty((nao, nao), dtype=torch.float64, device=D.device)
        opts = Opts(0, float(tau), 0, 0, 0, int(bool(deterministic)))
        _check(load_library().mderi_kbuild(self._h, basis._h, _vp(D.data_ptr()), _vp(out.data_ptr()), nao,
                                           ctypes.byref(opts), _stream_handle(stream)))
        return out

    def kernel_timing(self, enable: bool):
        """Brackets every fused-kernel launch with HIP events on its stream."""
        _check(load_library().mderi_kernel_timing(self._h, int(bool(enable))))

    def progress(self, enable: bool):
        """Prints a line to stderr as each launch group of the J/K builds and the gradient finishes."""
        _check(load_library().mderi_progress(self._h, int(bool(enable))))

    def tune_save(self, path):
        """Writes the autotuner's tile choices held by the context to `path`."""
        _check(load_library().mderi_tune_save(self._h, os.fsencode(path)))

    def tune_load(self, path):
        """Reads tile choices written by tune_save (same GPU architecture)."""
        _check(load_library().mderi_tune_load(self._h, os.fsencode(path)))

    def set_workspace_limit(self, nbytes: int):
        """Caps the context's device workspace (0 = no cap); releases what it holds."""
        _check(load_library().mderi_set_workspace_limit(self._h, int(nbytes)))

    def kernel_times(self):
        """Durations (ms) of the fused-kernel launches recorded since the last read."""
        n = ctypes.c_int(0)
        _check(load_library().mderi_kernel_times(self._h, None, 0, ctypes.byref(n)))
        buf = np.zeros(max(n.value, 1))
        _check(load_library().mderi_kernel_times(self._h, buf.ctypes.data_as(_dp), len(buf), ctypes.byref(n)))
        return buf[:n.value].copy()

    def kbuild_grad(self, basis: "Basis", Wl, natom, Wr=None, pattern=EXCHANGE, scale=1.0, tau=1e-12, out=None,
                    accumulate=False, symmetric=None, stream=None, deterministic=False):
        """dE/dR of E = scale sum W_abcd (ab|cd) with W = Wl_ac Wr_bd (pattern
        EXCHANGE; Wl = Wr = D gives tr(D K[D])) or Wl_ab Wr_cd (COULOMB), W
        held fixed -> torch float64 [natom, 3] (atoms as mapped by the basis'
        atom list).  Wr defaults to Wl; symmetric (default: Wr is None, the
        density case) declares Wl = Wr symmetric (MDERI_FLAG_SYMMETRIC).
        deterministic: fixed-point integer accumulation, the same bits on every run."""
        import torch
        nao = basis.nao()
        if symmetric is None:
            symmetric = Wr is None
        Wr = Wl if Wr is None else Wr
        for W in (Wl, Wr):
            assert W.dtype == torch.float64 and W.is_cuda and W.shape == (nao, nao)
        Wl, Wr = Wl.contiguous(), Wr.contiguous()
        if out is None:
            out = torch.zeros((natom, 3), dtype=torch.float64, device=Wl.device)
        opts = Opts(0, float(tau), FLAG_SYMMETRIC if (symmetric and Wr is Wl) else 0, 0, 0, int(bool(deterministic)))
        _check(load_library().mderi_kbuild_grad(self._h, basis._h, int(pattern), _vp(Wl.data_ptr()),
                                                _vp(Wr.data_ptr()), nao, float(scale), _vp(out.data_ptr()),
                                                int(natom), int(bool(accumulate)), ctypes.byref(opts),
                                                _stream_handle(stream)))
        return out

    def schwarz(self, basis: "Basis", pairs, stream=None):
        """Schwarz factors Q_ij = sqrt(max |(ab|ab)|) -> torch float64 tensor [npair]."""
        import torch
        pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        Q = torch.empty(max(len(pairs), 1), dtype=torch.float64, device=f"cuda:{self.device}")
        _check(load_library().mderi_schwarz(self._h, basis._h, len(pairs), pairs.ctypes.data_as(_ip),
                                            _vp(Q.data_ptr()), _stream_handle(stream)))
        return Q[:len(pairs)]


class Basis:
    """A shell list uploaded to the device (see include/mderi.h)."""

    def __init__(self, ctx: Context, l, nprim, exps, coefs, centers, atom=None, normalize=1):
        self.ctx = ctx
        self.l = np.ascontiguousarray(l, dtype=np.int32)
        self.nprim = np.ascontiguousarray(nprim, dtype=np.int32)
        self.exps = np.ascontiguousarray(exps, dtype=np.float64)
        self.coefs = np.ascontiguousarray(coefs, dtype=np.float64)
        self.centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        self.atom = None if atom is None else np.ascontiguousarray(atom, dtype=np.int32)
        h = _vp()
        _check(load_library().mderi_basis_upload(
            ctx._h, len(self.l), self.l.ctypes.data_as(_ip), self.nprim.ctypes.data_as(_ip),
            self.exps.ctypes.data_as(_dp), self.coefs.ctypes.data_as(_dp), self.centers.ctypes.data_as(_dp),
            None if self.atom is None else self.atom.ctypes.data_as(_ip), int(normalize), ctypes.byref(h)))
        self._h = h

    @property
    def nshell(self):
        return len(self.l)

    def pair_dim(self, pairs):
        """N(l_a) N(l_b) of the first pair, or None if it indexes outside the basis."""
        if len(pairs) == 0 or pairs.min() < 0 or pairs.max() >= len(self.l):
            return None
        return nsph(int(self.l[pairs[0, 0]])) * nsph(int(self.l[pairs[0, 1]]))

    def nao(self):
        return int(load_library().mderi_basis_nao(self._h))

    def set_centers(self, centers, stream=None):
        """Moves the shells to centers (torch float64 [nshell, 3] on the
        device), copied on the stream; the tensor must stay alive until the
        stream reaches the copy."""
        import torch
        assert centers.dtype == torch.float64 and centers.is_cuda and centers.shape == (self.nshell, 3)
        assert centers.is_contiguous()
        _check(load_library().mderi_basis_set_centers(self._h, _vp(centers.data_ptr()), _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load_library().mderi_basis_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exchange_energy(ctx: Context, coords, D, basis: "Basis", tau=1e-12):
    """E = tr(D K[D]) as a differentiable function of atom coordinates
    coords [natom, 3] (bohr) and the symmetric density D [nao, nao] (both
    float64 on the device).  `basis` is an uploaded Basis with an atom map;
    its shells are moved to coords[atom] on the device (mderi_basis_set_centers)
    before the build.  Forward: E from mderi_jkbuild; backward: dE/dcoords
    from mderi_kbuild_grad, dE/dD = 2 K."""
    return _ExchangeEnergy.apply(coords, D, ctx, basis, float(tau))


def _make_exchange_function():
    import torch

    class ExchangeEnergy(torch.autograd.Function):
        @staticmethod
        def forward(fctx, coords, D, ctx, basis, tau):
            atom = torch.as_tensor(basis.atom, dtype=torch.long, device=coords.device)
            centers = coords.detach()[atom].contiguous()
            basis.set_centers(centers)
            _, K, E = ctx.jkbuild(basis, D.detach(), want_j=False, tau=tau, energies=True)
            fctx.ctx, fctx.basis, fctx.tau, fctx.natom = ctx, basis, tau, coords.shape[0]
            fctx.save_for_backward(D.detach(), K, centers)
            return E[1]

        @staticmethod
        def backward(fctx, gE):
            D, K, centers = fctx.saved_tensors
            gc = gD = None
            if fctx.needs_input_grad[0]:
                fctx.basis.set_centers(centers)
                gc = gE * fctx.ctx.kbuild_grad(fctx.basis, D, fctx.natom, tau=fctx.tau)
            if fctx.needs_input_grad[1]:
                gD = 2.0 * gE * K
            return gc, gD, None, None, None

    return ExchangeEnergy


class _Lazy:
    def __init__(self):
        self._f = None

    def apply(self, *args):
        if self._f is None:
            self._f = _make_exchange_function()
        return self._f.apply(*args)


_ExchangeEnergy = _Lazy()
