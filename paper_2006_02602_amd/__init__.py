"""MI355X cavity library: Python binding of libcavity.so (include/cavity.h).

The functions below carry the C ABI's names and only marshal arguments:
torch tensors provide device memory and the current HIP stream, every step
of the computation runs in the library's HIP kernels.  Nothing here falls
back to a CPU implementation; if the library is missing, the first call
raises ImportError.

The solver is the explicit pseudo-time sweep of the 3D buoyancy-driven
cavity of Xue & Roy (arXiv:2006.02602, Sec. 2-3) with the in-device halo
pack/unpack of its "Optimized V1-V3" versions (Sec. 4.5).
"""
import ctypes
import weakref
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

from ._lib import (CAV_EHIP, CAV_EINVAL, CAV_ENONFINITE, CAV_ENOSYS, CAV_ESIZE, CAV_F32, CAV_F64, CAV_OK,
                   EXPORTS, CavBatch, CavBatchMember, CavError, CavGrid, CavHalo, CavKernelTime, CavLayout,
                   CavParams, check, lib)

NG = 2
FIELDS = ("p", "u", "v", "w", "T")


@dataclass(frozen=True)
class Grid:
    ni: int
    nj: int
    nk: int
    ng: int = NG
    dtype: int = CAV_F64

    @staticmethod
    def cube(n: int, dtype: int = CAV_F64) -> "Grid":
        return Grid(n, n, n, NG, dtype)

    @property
    def torch_dtype(self):
        import torch
        return torch.float32 if self.dtype == CAV_F32 else torch.float64

    def c(self) -> CavGrid:
        return CavGrid(self.ni, self.nj, self.nk, self.ng, self.dtype)

    @property
    def shape(self) -> Tuple[int, int, int, int]:
        return (5, self.nk + 2 * self.ng, self.nj + 2 * self.ng, self.ni + 2 * self.ng)

    @property
    def ncell(self) -> int:
        return self.ni * self.nj * self.nk


@dataclass(frozen=True)
class Params:
    """Nondimensional problem parameters (Sec. 2); see include/cavity.h."""
    Ra: float = 1e3
    Pr: float = 0.71
    cfl: float = 0.5
    eps4: float = 1.0 / 16
    kappa: float = 0.25
    u_ref: float = 1.0
    t_hot: float = 1.0
    t_cold: float = 0.0
    t_inf: float = 0.5
    # None, or a float64 GPU tensor of nj*nk hot-wall temperatures (j fastest)
    t_hot_field: object = field(default=None, compare=False)

    def c(self) -> CavParams:
        f = self.t_hot_field
        if f is not None:
            import torch
            if not (f.is_cuda and f.dtype == torch.float64 and f.is_contiguous()):
                raise ValueError("t_hot_field must be a contiguous float64 GPU tensor")
            f = f.data_ptr()
        return CavParams(self.Ra, self.Pr, self.cfl, self.eps4, self.kappa, self.u_ref,
                         self.t_hot, self.t_cold, self.t_inf, f)


@dataclass(frozen=True)
class Halo:
    """Virtual split (Pi, Pj, Pk) and ghost width per field p, u, v, w, T."""
    split: Tuple[int, int, int] = (2, 2, 2)
    width: Tuple[int, int, int, int, int] = (1, 2, 2, 2, 2)

    def c(self) -> CavHalo:
        return CavHalo((ctypes.c_int32 * 3)(*self.split), (ctypes.c_int32 * 5)(*self.width))


def _ptr(t):
    """Device pointer and byte size of a tensor (or (ptr, nbytes) pair)."""
    if t is None:
        return None, 0
    if isinstance(t, tuple):
        return t
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr(), t.numel() * t.element_size()


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _grid(g):
    return g.c() if isinstance(g, Grid) else g


def _halo(h):
    if h is None:
        return None
    return h.c() if isinstance(h, Halo) else h


def _params(p):
    return p.c() if isinstance(p, Params) else p


# ---- the C ABI, name for name ------------------------------------------------

def cavity_layout(grid) -> CavLayout:
    out = CavLayout()
    check(lib().cavity_layout(ctypes.byref(_grid(grid)), ctypes.byref(out)))
    return out


def state_view(grid, q):
    """(5, nk+4, nj+4, ni+4) strided view of a flat state tensor in the
    library layout (cells and ghosts; the row padding is skipped)."""
    import torch
    g = grid if isinstance(grid, Grid) else Grid(grid.ni, grid.nj, grid.nk, grid.ng, grid.dtype)
    L = cavity_layout(g)
    return torch.as_strided(q, (5, g.nk + 2 * g.ng, g.nj + 2 * g.ng, g.ni + 2 * g.ng),
                            (L.sf, L.sk, L.sj, 1), q.storage_offset() + L.lead - g.ng)


def cavity_state_elems(grid) -> int:
    return int(lib().cavity_state_elems(ctypes.byref(_grid(grid))))


# Tile widths of the batched kernel per element type, (wide, narrow); the
# tile has 512 (FP64) or 256 (FP32) threads, so its height follows.
BATCH_TILE_WIDTHS = {CAV_F64: (64, 32), CAV_F32: (32, 16)}


def batch_tile(dtype: int, ti: int = 0):
    """(columns along i, rows along j) of the batched tile of width ti (0 =
    the wide shape) for element type dtype."""
    wide, narrow = BATCH_TILE_WIDTHS[dtype]
    w = narrow if ti == narrow else wide
    return w, (256 if dtype == CAV_F32 else 512) // w


def cavity_workspace_bytes(grid) -> int:
    return int(lib().cavity_workspace_bytes(ctypes.byref(_grid(grid))))


def halo_buffer_bytes(grid, halo) -> int:
    return int(lib().halo_buffer_bytes(ctypes.byref(_grid(grid)), ctypes.byref(_halo(halo))))


def cavity_init(grid, params, seed: int, noise_amp: float, q, stream=None) -> None:
    qp, _ = _ptr(q)
    check(lib().cavity_init(ctypes.byref(_grid(grid)), ctypes.byref(_params(params)),
                            ctypes.c_uint64(seed), float(noise_amp), qp, _stream(stream)))


def cavity_step(grid, params, halo, q, q_tmp, ws, halo_buf, nsteps: int, stream=None) -> None:
    qp, _ = _ptr(q)
    tp, _ = _ptr(q_tmp)
    wp, wb = _ptr(ws)
    bp, bb = _ptr(halo_buf)
    h = _halo(halo)
    check(lib().cavity_step(ctypes.byref(_grid(grid)), ctypes.byref(_params(params)),
                            ctypes.byref(h) if h is not None else None, qp, tp, wp, wb, bp, bb,
                            int(nsteps), _stream(stream)))


def cavity_step_from(grid, params, q_in, q_out, ws=None, stream=None) -> None:
    """One step out of place: q_out = step(q_in) (no halo); norms into ws
    when given."""
    ip, _ = _ptr(q_in)
    op, _ = _ptr(q_out)
    wp, wb = _ptr(ws)
    check(lib().cavity_step_from(ctypes.byref(_grid(grid)), ctypes.byref(_params(params)), ip, op, wp, wb,
                                 _stream(stream)))


def cavity_step_noalloc(grid, params, halo, q, q_tmp, halo_buf, norms, nsteps: int, stream=None) -> None:
    """cavity_step with its norm partials in the library's static device
    array (no workspace; the call allocates nothing).  norms: a device
    tensor of 5 float64 written with the last step's residual norms, or
    None to skip them."""
    qp, _ = _ptr(q)
    tp, _ = _ptr(q_tmp)
    bp, bb = _ptr(halo_buf)
    npt, nb = _ptr(norms)
    if npt is not None and nb < 5 * 8:
        raise ValueError("norms must hold 5 float64 values")
    h = _halo(halo)
    check(lib().cavity_step_noalloc(ctypes.byref(_grid(grid)), ctypes.byref(_params(params)),
                                    ctypes.byref(h) if h is not None else None, qp, tp, bp, bb, npt,
                                    int(nsteps), _stream(stream)))


def cavity_step_overlap(grid, params, halo, q, q_tmp, ws, halo_buf, nsteps: int, stream=None,
                        comm_stream=None) -> None:
    """cavity_step with the interior sweep overlapping the exchange on
    comm_stream (default: the same stream)."""
    qp, _ = _ptr(q)
    tp, _ = _ptr(q_tmp)
    wp, wb = _ptr(ws)
    bp, bb = _ptr(halo_buf)
    h = _halo(halo)
    s = _stream(stream)
    cs = s if comm_stream is None else _stream(comm_stream)
    check(lib().cavity_step_overlap(ctypes.byref(_grid(grid)), ctypes.byref(_params(params)),
                                    ctypes.byref(h) if h is not None else None, qp, tp, wp, wb, bp, bb,
                                    int(nsteps), s, cs))


def cavity_stream_copy(grid, q, q_tmp, stream=None) -> None:
    """The sweep's memory streams without its work (measurement support):
    copies the interior cells of q into q_tmp with the sweep's tiling."""
    qp, _ = _ptr(q)
    tp, _ = _ptr(q_tmp)
    check(lib().cavity_stream_copy(ctypes.byref(_grid(grid)), qp, tp, _stream(stream)))


def cavity_selftest_math(x, out, stream=None) -> None:
    """Test support: out[2m], out[2m+1] = the kernels' sqrt(x[m]), 1/x[m]."""
    xp, xb = _ptr(x)
    op, ob = _ptr(out)
    n = xb // 8
    if ob < 16 * n:
        raise ValueError("out must hold 2 * len(x) float64 values")
    check(lib().cavity_selftest_math(xp, op, n, _stream(stream)))


def halo_pack(grid, halo, q, buf, stream=None) -> None:
    qp, _ = _ptr(q)
    bp, bb = _ptr(buf)
    check(lib().halo_pack(ctypes.byref(_grid(grid)), ctypes.byref(_halo(halo)), qp, bp, bb,
                          _stream(stream)))


def halo_unpack(grid, halo, buf, q, stream=None) -> None:
    qp, _ = _ptr(q)
    bp, bb = _ptr(buf)
    check(lib().halo_unpack(ctypes.byref(_grid(grid)), ctypes.byref(_halo(halo)), bp, bb, qp,
                            _stream(stream)))


def cavity_residual_norm(grid, ws, stream=None):
    """The last step's residual L2 norms (p, u, v, w, T) as a list of floats."""
    wp, wb = _ptr(ws)
    out = (ctypes.c_double * 5)()
    check(lib().cavity_residual_norm(ctypes.byref(_grid(grid)), wp, wb, out, _stream(stream)))
    return [out[i] for i in range(5)]


def cavity_nusselt(grid, params, q, ws, stream=None) -> float:
    """Mean hot-wall Nusselt number of state q (FP64 accumulation)."""
    qp, _ = _ptr(q)
    wp, wb = _ptr(ws)
    out = ctypes.c_double(0.0)
    check(lib().cavity_nusselt(ctypes.byref(_grid(grid)), ctypes.byref(_params(params)), qp, wp, wb,
                               ctypes.byref(out), _stream(stream)))
    return out.value


def cavity_adjoint_workspace_bytes(grid) -> int:
    return int(lib().cavity_adjoint_workspace_bytes(ctypes.byref(_grid(grid))))


def cavity_nusselt_adjoint(grid, params, lam, dj_dthot, stream=None) -> None:
    check(lib().cavity_nusselt_adjoint(ctypes.byref(_grid(grid)), ctypes.byref(_params(params)), _ptr(lam)[0],
                                       _ptr(dj_dthot)[0], _stream(stream)))


def cavity_adjoint_step(grid, params, q_n, lam_in, lam_out, ws, dj_dthot, dj_dra, stream=None) -> None:
    ptrs = [_ptr(t)[0] for t in (q_n, lam_in, lam_out)]
    wp, wb = _ptr(ws)
    check(lib().cavity_adjoint_step(ctypes.byref(_grid(grid)), ctypes.byref(_params(params)),
                                    ptrs[0], ptrs[1], ptrs[2], wp, wb, _ptr(dj_dthot)[0],
                                    _ptr(dj_dra)[0], _stream(stream)))


def _members(members):
    arr = (CavBatchMember * len(members))()
    for i, m in enumerate(members):
        arr[i] = m
    return arr


def cavity_batch_table_bytes(members) -> int:
    return int(lib().cavity_batch_table_bytes(len(members), _members(members)))


def cavity_batch_build(members, table, stream=None) -> CavBatch:
    tp, tb = _ptr(table)
    out = CavBatch()
    check(lib().cavity_batch_build(len(members), _members(members), tp, tb, ctypes.byref(out), _stream(stream)))
    return out


def cavity_batch_step(batch: CavBatch, nsteps: int, nblocks: int = 0, stream=None) -> None:
    check(lib().cavity_batch_step(ctypes.byref(batch), int(nsteps), int(nblocks), _stream(stream)))


def cavity_batch_graph_create(batch: CavBatch, nsteps: int, nblocks: int = 0, stream=None):
    h = ctypes.c_void_p()
    check(lib().cavity_batch_graph_create(ctypes.byref(batch), int(nsteps), int(nblocks), _stream(stream),
                                          ctypes.byref(h)))
    return h.value


def cavity_batch_graph_launch(batch: CavBatch, graph_exec, stream=None) -> None:
    check(lib().cavity_batch_graph_launch(ctypes.byref(batch), graph_exec, _stream(stream)))


def cavity_batch_graph_destroy(graph_exec) -> None:
    check(lib().cavity_batch_graph_destroy(graph_exec))


def cavity_last_error() -> str:
    return lib().cavity_last_error().decode(errors="replace")


def cavity_timing_enable(on: bool) -> None:
    check(lib().cavity_timing_enable(1 if on else 0))


def cavity_timing_read():
    """{kernel name: (launches, total ms)} recorded since the last read."""
    arr = (CavKernelTime * 32)()
    n = ctypes.c_int32(0)
    check(lib().cavity_timing_read(arr, 32, ctypes.byref(n)))
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms))
            for i in range(min(n.value, 32))}


# ---- convenience: buffers for one cavity ------------------------------------

class Cavity:
    """Allocates the state, scratch state, workspace and halo buffer of one
    cavity with torch and drives the C ABI on the current stream."""

    def __init__(self, grid: Grid, params: Params = Params(), halo: Optional[Halo] = None,
                 device: str = "cuda"):
        import torch
        self.grid, self.params, self.halo = grid, params, halo
        n = cavity_state_elems(grid)
        if n == 0:
            raise CavError(CAV_EINVAL, cavity_last_error())
        self.q = torch.zeros(n, dtype=grid.torch_dtype, device=device)
        self.q_tmp = torch.zeros(n, dtype=grid.torch_dtype, device=device)
        self.ws = torch.zeros(cavity_workspace_bytes(grid) // 8, dtype=torch.float64, device=device)
        nb = halo_buffer_bytes(grid, halo) if halo is not None else 0
        es = 4 if grid.dtype == CAV_F32 else 8
        self.buf = torch.zeros(max(1, nb // es), dtype=grid.torch_dtype, device=device) if halo is not None else None

    def init(self, seed: int, noise_amp: float = 1e-3) -> "Cavity":
        cavity_init(self.grid, self.params, seed, noise_amp, self.q)
        return self

    def step(self, nsteps: int) -> "Cavity":
        cavity_step(self.grid, self.params, self.halo, self.q, self.q_tmp, self.ws, self.buf, nsteps)
        return self

    def step_overlap(self, nsteps: int, comm_stream=None) -> "Cavity":
        """Steps with the interior/exterior split; the exchange runs on
        comm_stream (a torch.cuda.Stream) when given."""
        cavity_step_overlap(self.grid, self.params, self.halo, self.q, self.q_tmp, self.ws, self.buf, nsteps,
                            comm_stream=comm_stream)
        return self

    def norms(self):
        return cavity_residual_norm(self.grid, self.ws)

    def nusselt(self) -> float:
        return cavity_nusselt(self.grid, self.params, self.q, self.ws)

    def fields(self, which=None):
        """A state as a (5, nk+4, nj+4, ni+4) strided view (default: q)."""
        return state_view(self.grid, self.q if which is None else which)

    def interior(self):
        g = self.grid.ng
        return self.fields()[:, g:g + self.grid.nk, g:g + self.grid.nj, g:g + self.grid.ni]


class Batch:
    """Many independent cavities advanced together (the batched form): one
    persistent launch per step over all members; optional graph replay.

    members: list of (Grid, Params), (Grid, Params, kc) or
    (Grid, Params, kc, ti) with ti the tile width: 0 = the wide shape; FP64
    64 (64 x 8) or 32 (32 x 16); FP32 32 (32 x 8) or 16 (16 x 16)."""

    def __init__(self, members, device: str = "cuda"):
        import torch
        self.grids, self.params, self.kcs = [], [], []
        self.q, self.q_tmp, self.ws = [], [], []
        cm = []
        for m in members:
            g, p = m[0], m[1]
            kc = m[2] if len(m) > 2 else 0
            ti = m[3] if len(m) > 3 else 0
            n = cavity_state_elems(g)
            if n == 0:
                raise CavError(CAV_EINVAL, cavity_last_error())
            q = torch.zeros(n, dtype=g.torch_dtype, device=device)
            qt = torch.zeros(n, dtype=g.torch_dtype, device=device)
            wb = cavity_workspace_bytes(g)
            ws = torch.zeros(wb // 8, dtype=torch.float64, device=device)
            self.grids.append(g)
            self.params.append(p)
            self.kcs.append(kc)
            self.q.append(q)
            self.q_tmp.append(qt)
            self.ws.append(ws)
            cm.append(CavBatchMember(g.c(), p.c(), q.data_ptr(), qt.data_ptr(), ws.data_ptr(), wb, kc, ti))
        self._members = cm
        nb = cavity_batch_table_bytes(cm)
        if nb == 0:
            raise CavError(CAV_EINVAL, "invalid batch members")
        self.table = torch.zeros(nb, dtype=torch.uint8, device=device)
        self.handle = cavity_batch_build(cm, self.table)
        self._graphs = weakref.WeakSet()

    def __len__(self):
        return len(self.grids)

    def retile(self, shapes) -> "Batch":
        """Rebuild the work list with (kc, ti) per member, keeping every
        member's state, workspace and the parity.  A graph captured from the
        old work list would replay it on the new table, so live graphs of
        this batch must be destroyed first."""
        import torch
        if any(gr.exec for gr in list(self._graphs)):
            raise CavError(CAV_EINVAL, "destroy this batch's graphs before retiling it")
        cm = [CavBatchMember(m.grid, m.params, m.q, m.q_tmp, m.ws, m.ws_bytes, int(kc), int(ti))
              for m, (kc, ti) in zip(self._members, shapes)]
        nb = cavity_batch_table_bytes(cm)
        if nb == 0:
            raise CavError(CAV_EINVAL, "invalid batch members")
        if nb > self.table.numel():
            self.table = torch.zeros(nb, dtype=torch.uint8, device=self.table.device)
        parity = self.handle.parity
        self.handle = cavity_batch_build(cm, self.table)
        self.handle.parity = parity
        self._members = cm
        self.kcs = [int(kc) for kc, _ in shapes]
        return self

    @property
    def cells(self) -> int:
        return int(self.handle.cells)

    def init(self, seeds, noise_amp: float = 1e-3) -> "Batch":
        """Seed every member (cavity_init on its q); the batch restarts at parity 0."""
        for g, p, q, s in zip(self.grids, self.params, self.q, seeds):
            cavity_init(g, p, int(s), noise_amp, q)
        self.handle.parity = 0
        return self

    def step(self, nsteps: int, nblocks: int = 0, stream=None) -> "Batch":
        cavity_batch_step(self.handle, nsteps, nblocks, stream)
        return self

    def state(self, m: int):
        """Flat tensor that holds member m's newest state."""
        return self.q_tmp[m] if self.handle.parity else self.q[m]

    def fields(self, m: int):
        return state_view(self.grids[m], self.state(m))

    def norms(self, m: int):
        return cavity_residual_norm(self.grids[m], self.ws[m])

    def graph(self, nsteps: int, nblocks: int = 0, stream=None) -> "BatchGraph":
        return BatchGraph(self, nsteps, nblocks, stream)


class BatchGraph:
    """An instantiated HIP graph of `nsteps` (even) batch steps."""

    def __init__(self, batch: Batch, nsteps: int, nblocks: int, stream):
        self.batch = batch
        self.exec = cavity_batch_graph_create(batch.handle, nsteps, nblocks, stream)
        batch._graphs.add(self)

    def launch(self, stream=None) -> None:
        cavity_batch_graph_launch(self.batch.handle, self.exec, stream)

    def destroy(self) -> None:
        if self.exec:
            cavity_batch_graph_destroy(self.exec)
            self.exec = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


__all__ = ["Batch", "BatchGraph", "Grid", "Params", "Halo", "Cavity", "CavError", "FIELDS", "NG", "EXPORTS", "state_view",
           "CAV_OK", "CAV_EINVAL", "CAV_ESIZE", "CAV_EHIP", "CAV_ENONFINITE", "CAV_ENOSYS", "CAV_F64", "CAV_F32"] + list(EXPORTS)
