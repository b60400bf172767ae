"""Thin Python binding of libmdvrp (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels. PyTorch only
provides device memory (workspaces, input and output arrays) and the stream.
Importing works without a GPU; creating objects needs one and fails loudly
when the compiled library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdvrp.so")

OK, EINVAL, ERANGE, ENOSPC, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
FAM_RELOCATE, FAM_SWAP, FAM_2OPT_STAR, FAM_2OPT, FAM_DEPOT_INSERT, FAM_DEPOT_REPLACE = 1, 2, 4, 8, 16, 32
FAM_ALL = 0x3F
EVAL_FILTERED = 2
LS_PASSES, LS_UNION = 0, 1
FILTER_NONE, FILTER_LISTS, FILTER_MLP = 0, 1, 2
RESCORE_STEP, RESCORE_PASS = 0, 1
LAYOUT_AUTO, LAYOUT_GIVEN, LAYOUT_ORDERED = 0, 1, 2
MLP_PARAMS = 74497
TRAIN_STATIC_MAX_N = 4096  # samples per call of the allocation-free training step
PAIR_FAMILIES = FAM_RELOCATE | FAM_SWAP | FAM_2OPT_STAR | FAM_2OPT


class MdvrpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libmdvrp status {status}: {msg}")
        self.status = status


class InstanceDesc(C.Structure):
    _fields_ = [("n_depots", C.c_int32), ("n_customers", C.c_int32),
                ("c", C.c_void_p), ("t", C.c_void_p), ("q", C.c_void_p), ("s", C.c_void_p),
                ("e", C.c_void_p), ("l", C.c_void_p),
                ("Q", C.c_int32), ("NV", C.c_int32), ("Dmax", C.c_int32),
                ("open_routes", C.c_int32), ("has_tw", C.c_int32), ("theta", C.c_int32),
                ("w_tw", C.c_int32), ("w_load", C.c_int32), ("w_dur", C.c_int32), ("w_depot", C.c_int32),
                ("layout", C.c_int32)]


class Moves(C.Structure):
    """mdvrp_moves: device arrays of the improving-move list."""
    _fields_ = [("dF", C.c_void_p), ("dD", C.c_void_p), ("id", C.c_void_p), ("kind", C.c_void_p),
                ("variant", C.c_void_p), ("changed", C.c_void_p), ("unit", C.c_void_p), ("a", C.c_void_p),
                ("b", C.c_void_p), ("res", C.c_void_p), ("cap", C.c_int64), ("count", C.c_void_p)]


MOVE_FIELDS = [("dF", np.int64), ("dD", np.int64), ("id", np.uint64), ("kind", np.uint8), ("variant", np.uint8),
               ("changed", np.uint8), ("unit", np.int32), ("a", np.int32), ("b", np.int32), ("res", np.int32, (3,))]
MOVE_DTYPE = np.dtype(MOVE_FIELDS)


class LsOptions(C.Structure):
    _fields_ = [("mode", C.c_int32), ("leader_only", C.c_int32), ("max_passes", C.c_int32),
                ("poll_every", C.c_int32), ("seed", C.c_uint64), ("filter", C.c_int32), ("rescore", C.c_int32),
                ("mlp", C.c_void_p), ("graph", C.c_int32), ("penalty_adapt", C.c_int32),
                ("w_min", C.c_int32 * 4), ("w_max", C.c_int32 * 4)]


class LsStats(C.Structure):
    _fields_ = [("passes", C.c_int64), ("steps", C.c_int64), ("moves_applied", C.c_int64),
                ("evaluated", C.c_int64), ("F", C.c_int64), ("fallback_passes", C.c_int64),
                ("device_ms", C.c_double), ("converged", C.c_int32), ("err", C.c_int32),
                ("w_final", C.c_int64 * 4)]


DENSE_DTYPE = np.dtype([("dF", np.int64), ("dD", np.int64), ("dTW", np.int64), ("dLX", np.int64),
                        ("dDX", np.int64), ("dV4", np.int64), ("id", np.uint64), ("unit", np.int32),
                        ("res", np.int32, (3,))])
assert DENSE_DTYPE.itemsize == 72

_lib = None

EXPORTED = [
    "mdvrp_validate_instance_host", "mdvrp_instance_workspace_query", "mdvrp_instance_create",
    "mdvrp_instance_info", "mdvrp_instance_copy_lists", "mdvrp_instance_destroy",
    "mdvrp_batch_workspace_query", "mdvrp_batch_create", "mdvrp_batch_destroy",
    "mdvrp_validate_solutions_host", "mdvrp_solutions_load", "mdvrp_solutions_export", "mdvrp_batch_cost",
    "mdvrp_batch_state", "mdvrp_eval_neighbourhood", "mdvrp_eval_dense", "mdvrp_select_multimove",
    "mdvrp_apply_moves",
    "mdvrp_local_search_to_optimum", "mdvrp_status_string", "mdvrp_last_error", "mdvrp_family_order",
    "mdvrp_profile_enable", "mdvrp_profile_sampling", "mdvrp_profile_read", "mdvrp_eval_footprint",
    "mdvrp_mlp_workspace_query", "mdvrp_mlp_create", "mdvrp_mlp_params", "mdvrp_mlp_sync", "mdvrp_mlp_destroy",
    "mdvrp_mlp_act_bytes", "mdvrp_mlp_forward", "mdvrp_mlp_backward", "mdvrp_mlp_bce", "mdvrp_adam_step",
    "mdvrp_mlp_train_step", "mdvrp_mlp_train_step_static", "mdvrp_filter_workspace_query", "mdvrp_filter_attach",
    "mdvrp_filter_anchor_count",
    "mdvrp_filter_features", "mdvrp_filter_labels", "mdvrp_filter_score_topk", "mdvrp_filter_eta_lists",
    "mdvrp_filter_export", "mdvrp_autotune", "mdvrp_set_tile_shapes",
    "mdvrp_population_workspace_query", "mdvrp_population_distance", "mdvrp_population_reduce",
    "mdvrp_solutions_load_partial", "mdvrp_repair",
    "mdvrp_dcrex_workspace_query", "mdvrp_dcrex_counts", "mdvrp_dcrex_pick", "mdvrp_ucb_select", "mdvrp_ucb_update",
]
REPAIR_FBI, REPAIR_IBI, REPAIR_FRI, REPAIR_IRI, REPAIR_RI = range(5)
PROF_CLASSES = ["eval_pairs", "eval_depot_insert", "eval_depot_replace", "select", "apply", "filter_score"]
STATE_WORDS = 16


def lib():
    """Load libmdvrp.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (paper_2605_05208_amd.build)")
        L = C.CDLL(LIB_PATH)
        p, i32, i64, u32, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_size_t
        sig = {
            "mdvrp_validate_instance_host": [p],
            "mdvrp_instance_workspace_query": [p, p],
            "mdvrp_instance_create": [p, p, sz, p, p],
            "mdvrp_instance_info": [p, p],
            "mdvrp_instance_copy_lists": [p, p, p, p],
            "mdvrp_batch_workspace_query": [p, i32, p, i32, p],
            "mdvrp_batch_create": [p, i32, p, i32, p, sz, p, p],
            "mdvrp_validate_solutions_host": [p, i32, p, i32, p, p, p, p, p],
            "mdvrp_solutions_load": [p, p, p, p, p, p, i32, i32, p],
            "mdvrp_solutions_export": [p, p, p, p, p, p, p],
            "mdvrp_batch_cost": [p, p, p, p],
            "mdvrp_batch_state": [p, p],
            "mdvrp_eval_neighbourhood": [p, u32, p, i32, p, u32, p, p],
            "mdvrp_eval_dense": [p, u32, u32, p, i64, p, p],
            "mdvrp_select_multimove": [p, u32, i32, p, p, p, i32, p],
            "mdvrp_apply_moves": [p, p],
            "mdvrp_local_search_to_optimum": [p, p, p, p],
            "mdvrp_family_order": [i32, u64, i64, p],
            "mdvrp_profile_enable": [p, u32, i32],
            "mdvrp_profile_sampling": [p, i32],
            "mdvrp_profile_read": [p, p, p],
            "mdvrp_eval_footprint": [p, u32, p, i64, p],
            "mdvrp_mlp_workspace_query": [p],
            "mdvrp_mlp_create": [p, sz, p, p, p],
            "mdvrp_mlp_params": [p, p],
            "mdvrp_mlp_sync": [p, i32, p],
            "mdvrp_mlp_act_bytes": [i32, p],
            "mdvrp_mlp_forward": [p, p, i32, p, p, sz, p],
            "mdvrp_mlp_backward": [p, p, p, i32, p, p, sz, p],
            "mdvrp_mlp_bce": [p, p, p, p, i32, p, p, p],
            "mdvrp_adam_step": [p, p, C.c_float, i32, p],
            "mdvrp_mlp_train_step": [p, p, p, p, i32, C.c_float, i32, p, p, p, p, sz, p],
            "mdvrp_mlp_train_step_static": [p, p, p, p, i32, C.c_float, i32, p, p, p, p],
            "mdvrp_population_workspace_query": [p, p, i32, p],
            "mdvrp_population_distance": [p, p, i32, p, p, p, p, sz, p],
            "mdvrp_population_reduce": [p, p, i32, i32, C.c_double, i32, p, p, p, p, p],
            "mdvrp_solutions_load_partial": [p, p, p, p, p, p, i32, i32, p],
            "mdvrp_repair": [p, i32, u64, p, p, p],
            "mdvrp_dcrex_workspace_query": [i32, i32, i32, i32, p],
            "mdvrp_dcrex_counts": [i32, i32, i32, i32, p, p, p, p, p, i32, i32, p, p, p, p, p, p, p, p, p, sz, p],
            "mdvrp_dcrex_pick": [i32, i32, p, p, p, p, u64, p, p],
            "mdvrp_ucb_select": [i32, p, p, p, p],
            "mdvrp_ucb_update": [i32, p, p, p, p, C.c_double, p],
            "mdvrp_filter_workspace_query": [p, i32, p],
            "mdvrp_filter_attach": [p, i32, p, sz, p],
            "mdvrp_filter_anchor_count": [p, p],
            "mdvrp_filter_features": [p, p, p],
            "mdvrp_filter_labels": [p, u32, p, p],
            "mdvrp_filter_score_topk": [p, p, p, p],
            "mdvrp_filter_eta_lists": [p, p],
            "mdvrp_filter_export": [p, p, p],
            "mdvrp_autotune": [p, u32, i32, p, p],
            "mdvrp_set_tile_shapes": [p, p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.mdvrp_instance_destroy.argtypes = [p]
        L.mdvrp_instance_destroy.restype = None
        L.mdvrp_batch_destroy.argtypes = [p]
        L.mdvrp_batch_destroy.restype = None
        L.mdvrp_mlp_destroy.argtypes = [p]
        L.mdvrp_mlp_destroy.restype = None
        L.mdvrp_status_string.argtypes = [i32]
        L.mdvrp_status_string.restype = C.c_char_p
        L.mdvrp_last_error.argtypes = []
        L.mdvrp_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(status):
    if status != OK:
        raise MdvrpError(status, lib().mdvrp_last_error().decode())
    return status


def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _dev_i32(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda")


def desc_from_host(inst) -> InstanceDesc:
    """Descriptor whose array pointers are host numpy arrays (for host validation)."""
    keep = [np.ascontiguousarray(x, dtype=np.int32) for x in (inst.c, inst.t, inst.q, inst.s, inst.e, inst.l)]
    d = InstanceDesc(inst.n_depots, inst.n_customers, *[k.ctypes.data for k in keep],
                     inst.Q, inst.NV, inst.Dmax, inst.open_routes, inst.has_tw, inst.theta,
                     inst.w_tw, inst.w_load, inst.w_dur, inst.w_depot, LAYOUT_AUTO)
    d._keep = keep
    return d


class Instance:
    """Device-resident instance (c, t, node arrays) plus its preprocessing."""

    def __init__(self, inst, layout=None):
        torch = _torch()
        self.inst = inst
        layout = LAYOUT_AUTO if layout is None else layout
        self.c = _dev_i32(inst.c)
        self.t = self.c if inst.t is inst.c else _dev_i32(inst.t)
        self.q, self.s, self.e, self.l = (_dev_i32(x) for x in (inst.q, inst.s, inst.e, inst.l))
        self.desc = InstanceDesc(inst.n_depots, inst.n_customers, self.c.data_ptr(), self.t.data_ptr(),
                                 self.q.data_ptr(), self.s.data_ptr(), self.e.data_ptr(), self.l.data_ptr(),
                                 inst.Q, inst.NV, inst.Dmax, inst.open_routes, inst.has_tw, inst.theta,
                                 inst.w_tw, inst.w_load, inst.w_dur, inst.w_depot, layout)
        nbytes = C.c_size_t(0)
        check(lib().mdvrp_instance_workspace_query(C.byref(self.desc), C.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        check(lib().mdvrp_instance_create(C.byref(self.desc), _dptr(self.ws), nbytes.value, _stream(), C.byref(h)))
        self.handle = h

    def info(self):
        out = np.zeros(8, np.int64)
        check(lib().mdvrp_instance_info(self.handle, out.ctypes.data_as(C.c_void_p)))
        keys = ["Theta", "gamma_num", "gamma_den", "w_depot", "max_c", "min_c", "max_t", "len_guard"]
        return dict(zip(keys, (int(x) for x in out)))

    def lists(self):
        torch = _torch()
        nc, th = self.inst.n_customers, self.inst.theta
        a = torch.empty(nc * th, dtype=torch.int32, device="cuda")
        b = torch.empty(nc, dtype=torch.int32, device="cuda")
        check(lib().mdvrp_instance_copy_lists(self.handle, _dptr(a), _dptr(b), _stream()))
        torch.cuda.synchronize()
        return a.cpu().numpy(), b.cpu().numpy()

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mdvrp_instance_destroy(h)
            self.handle = None


class Batch:
    """Units = (instance, solution); one solution per unit."""

    def __init__(self, instances, unit_inst):
        torch = _torch()
        self.instances = list(instances)
        self.unit_inst = np.ascontiguousarray(unit_inst, dtype=np.int32)
        self.n_units = len(self.unit_inst)
        arr = (C.c_void_p * len(self.instances))(*[i.handle.value for i in self.instances])
        self._arr = arr
        nbytes = C.c_size_t(0)
        check(lib().mdvrp_batch_workspace_query(arr, len(self.instances), self.unit_inst.ctypes.data_as(C.c_void_p),
                                                self.n_units, C.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        check(lib().mdvrp_batch_create(arr, len(self.instances), self.unit_inst.ctypes.data_as(C.c_void_p),
                                       self.n_units, _dptr(self.ws), nbytes.value, _stream(), C.byref(h)))
        self.handle = h
        self.nc = np.array([self.instances[i].inst.n_customers for i in self.unit_inst], np.int64)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mdvrp_batch_destroy(h)
            self.handle = None

    # ------------------------------------------------------------------ solutions
    def load(self, solutions):
        from .gen import batch_flat
        nodes, offs, st, en, so = batch_flat(solutions)
        self._in = [_dev_i32(x) for x in (nodes if len(nodes) else np.zeros(1, np.int32), offs, st, en, so)]
        n, o, s, e, u = self._in
        check(lib().mdvrp_solutions_load(self.handle, _dptr(n), _dptr(o), _dptr(s), _dptr(e), _dptr(u),
                                         len(st), len(nodes), _stream()))

    def load_partial(self, solutions):
        """Load solutions from which customers may be missing (for repair)."""
        from .gen import batch_flat
        nodes, offs, st, en, so = batch_flat(solutions)
        pad = lambda a: a if len(a) else np.zeros(1, np.int32)  # noqa: E731
        self._in = [_dev_i32(x) for x in (pad(nodes), offs, pad(st), pad(en), so)]
        n, o, s, e, u = self._in
        check(lib().mdvrp_solutions_load_partial(self.handle, _dptr(n), _dptr(o), _dptr(s), _dptr(e), _dptr(u),
                                                 len(st), len(nodes), _stream()))

    def repair(self, op, seed=0):
        """Insert the missing customers of every unit with operator op (REPAIR_*): per unit
        (inserted customers in insertion order, positions evaluated)."""
        torch = _torch()
        tot = int(self.nc.sum())
        order = torch.full((max(tot, 1),), -1, dtype=torch.int32, device="cuda")
        nev = torch.zeros(self.n_units, dtype=torch.int64, device="cuda")
        check(lib().mdvrp_repair(self.handle, int(op), int(seed), _dptr(order), _dptr(nev), _stream()))
        torch.cuda.synchronize()
        o = order.cpu().numpy()
        base = np.concatenate([[0], np.cumsum(self.nc)])
        out = []
        for k in range(self.n_units):
            seg = o[base[k]:base[k + 1]]
            out.append([int(v) for v in seg[seg >= 0]])
        return out, [int(v) for v in nev.cpu().numpy()]

    def export(self):
        from .gen import Solution
        torch = _torch()
        tot_n = int(self.nc.sum())
        tot_r = int((self.nc + 1).sum())
        nodes = torch.empty(max(tot_n, 1), dtype=torch.int32, device="cuda")
        offs = torch.empty(tot_r + 1, dtype=torch.int32, device="cuda")
        st = torch.empty(tot_r, dtype=torch.int32, device="cuda")
        en = torch.empty(tot_r, dtype=torch.int32, device="cuda")
        cnt = torch.empty(self.n_units, dtype=torch.int32, device="cuda")
        check(lib().mdvrp_solutions_export(self.handle, _dptr(nodes), _dptr(offs), _dptr(st), _dptr(en), _dptr(cnt),
                                           _stream()))
        torch.cuda.synchronize()
        nodes, offs, st, en, cnt = (x.cpu().numpy() for x in (nodes, offs, st, en, cnt))
        out = []
        rb = 0
        for k in range(self.n_units):
            routes = []
            for r in range(int(cnt[k])):
                a, b = int(offs[rb + r]), int(offs[rb + r + 1])
                routes.append((int(st[rb + r]), [int(x) for x in nodes[a:b]], int(en[rb + r])))
            out.append(Solution(routes))
            rb += int(self.nc[k]) + 1
        return out

    def cost(self):
        torch = _torch()
        F = torch.empty(self.n_units, dtype=torch.int64, device="cuda")
        T = torch.empty(self.n_units * 6, dtype=torch.int64, device="cuda")
        check(lib().mdvrp_batch_cost(self.handle, _dptr(F), _dptr(T), _stream()))
        torch.cuda.synchronize()
        return F.cpu().numpy(), T.cpu().numpy().reshape(self.n_units, 6)

    def state(self):
        out = np.zeros(self.n_units * STATE_WORDS, np.int64)
        check(lib().mdvrp_batch_state(self.handle, out.ctypes.data_as(C.c_void_p)))
        return out.reshape(self.n_units, STATE_WORDS)

    def load_device(self, nodes, offs, starts, ends, unit_route_off, n_routes, n_nodes):
        """Load from device tensors already resident in HBM (int32)."""
        check(lib().mdvrp_solutions_load(self.handle, _dptr(nodes), _dptr(offs), _dptr(starts), _dptr(ends),
                                         _dptr(unit_route_off), n_routes, n_nodes, _stream()))

    def profile_enable(self, class_mask=0x1F, max_launches=1 << 16):
        """Time the kernel classes in class_mask (bit k = PROF_CLASSES[k]); 0 turns timing off."""
        check(lib().mdvrp_profile_enable(self.handle, class_mask, max_launches))

    def profile_sampling(self, every: int):
        """Time only every n-th launch of each class (1 = all)."""
        check(lib().mdvrp_profile_sampling(self.handle, int(every)))

    def profile_read(self):
        n = np.zeros(8, np.int64)
        ms = np.zeros(8, np.float64)
        check(lib().mdvrp_profile_read(self.handle, n.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p)))
        return {name: (int(n[k]), float(ms[k])) for k, name in enumerate(PROF_CLASSES)}

    # ------------------------------------------------------------------ hot path
    def eval_neighbourhood(self, fam_mask=FAM_ALL, dense_cap=0, filtered=False, cand=None, moves_cap=0,
                           want_evaluated=False):
        """Evaluate the families of fam_mask. dense_cap > 0: every evaluated move as a
        DENSE_DTYPE array (mdvrp_eval_dense). Otherwise mdvrp_eval_neighbourhood with,
        optionally, caller candidate lists cand (int32 [n_customers of the batch, k], units
        in batch order), the improving-move list (moves_cap rows; MOVE_DTYPE array) and the
        per-unit evaluated counts. Returns (moves or None, evaluated or None) then."""
        torch = _torch()
        fl = EVAL_FILTERED if filtered else 0
        if dense_cap:
            rec = torch.empty(dense_cap * DENSE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            check(lib().mdvrp_eval_dense(self.handle, fam_mask, fl, _dptr(rec), dense_cap, _dptr(cnt), _stream()))
            torch.cuda.synchronize()
            n = int(cnt.item())
            if n > dense_cap:
                raise MdvrpError(ENOSPC, f"dense table needs {n} records")
            return np.frombuffer(rec[:n * DENSE_DTYPE.itemsize].cpu().numpy().tobytes(), dtype=DENSE_DTYPE)
        cand_t, k = None, 0
        if cand is not None:
            cand_np = np.ascontiguousarray(cand, dtype=np.int32)
            k = int(cand_np.shape[1])
            cand_t = torch.from_numpy(cand_np.ravel()).to("cuda")
        mv, arrs = None, None
        if moves_cap:
            cap = int(moves_cap)
            arrs = {name: torch.empty(cap * (3 if name == "res" else 1),
                                      dtype={np.int64: torch.int64, np.uint64: torch.int64, np.uint8: torch.uint8,
                                             np.int32: torch.int32}[dt], device="cuda")
                    for name, dt, *_ in MOVE_FIELDS}
            arrs["count"] = torch.zeros(1, dtype=torch.int64, device="cuda")
            mv = Moves(*[arrs[name].data_ptr() for name, *_ in MOVE_FIELDS], cap, arrs["count"].data_ptr())
        ev = torch.empty(self.n_units, dtype=torch.int64, device="cuda") if want_evaluated else None
        st = lib().mdvrp_eval_neighbourhood(self.handle, fam_mask, _dptr(cand_t) if cand_t is not None else None, k,
                                            C.byref(mv) if mv is not None else None, fl,
                                            _dptr(ev) if ev is not None else None, _stream())
        if st == ENOSPC and arrs is not None:
            raise MdvrpError(ENOSPC, f"move list needs {int(arrs['count'].item())} rows")
        check(st)
        out = None
        if arrs is not None:
            torch.cuda.synchronize()
            n = int(arrs["count"].item())
            out = np.zeros(n, MOVE_DTYPE)
            for name, dt, *shape in MOVE_FIELDS:
                a = arrs[name].cpu().numpy()
                if dt == np.uint64:
                    a = a.view(np.uint64)
                out[name] = a[:3 * n].reshape(n, 3) if name == "res" else a[:n]
        evn = ev.cpu().numpy() if ev is not None else None
        return out, evn

    def eval_footprint(self, fam_mask=FAM_ALL):
        """Distinct matrix entries (c/t) the evaluation of fam_mask reads, per instance."""
        torch = _torch()
        words = [(i.inst.N * i.inst.N + 31) // 32 for i in self.instances]
        bits = torch.zeros(sum(words), dtype=torch.int32, device="cuda")
        check(lib().mdvrp_eval_footprint(self.handle, fam_mask, _dptr(bits), sum(words), _stream()))
        b = bits.cpu().numpy().view(np.uint32)
        out, at = [], 0
        for w in words:
            out.append(int(np.unpackbits(b[at:at + w].view(np.uint8)).sum()))
            at += w
        return out

    def select_multimove(self, fam_mask=FAM_ALL, leader_only=0, want=True):
        torch = _torch()
        if not want:
            check(lib().mdvrp_select_multimove(self.handle, fam_mask, leader_only, None, None, None, 0, _stream()))
            return None
        cap = int(self.nc.max()) + 1
        ids = torch.empty(self.n_units * cap, dtype=torch.int64, device="cuda")
        dF = torch.empty(self.n_units * cap, dtype=torch.int64, device="cuda")
        cnt = torch.empty(self.n_units, dtype=torch.int32, device="cuda")
        check(lib().mdvrp_select_multimove(self.handle, fam_mask, leader_only, _dptr(ids), _dptr(dF), _dptr(cnt), cap,
                                           _stream()))
        torch.cuda.synchronize()
        ids = ids.cpu().numpy().view(np.uint64).reshape(self.n_units, cap)
        dF = dF.cpu().numpy().reshape(self.n_units, cap)
        cnt = cnt.cpu().numpy()
        return [(ids[k, :cnt[k]].copy(), dF[k, :cnt[k]].copy()) for k in range(self.n_units)]

    def apply_moves(self):
        check(lib().mdvrp_apply_moves(self.handle, _stream()))

    def local_search_to_optimum(self, mode=LS_PASSES, seed=0, max_passes=0, leader_only=0, poll_every=1,
                                filter=FILTER_NONE, mlp=None, rescore=RESCORE_STEP, graph=False, adapt=None):
        """adapt = (w_min, w_max), four weights each (time window, load, duration, depot):
        dynamic penalty coefficients within those bounds; None = the current fixed weights."""
        opt = LsOptions(mode, leader_only, max_passes, poll_every, seed, filter, rescore,
                        mlp.handle.value if mlp is not None else None, 1 if graph else 0, 0)
        if adapt is not None:
            opt.penalty_adapt = 1
            opt.w_min = (C.c_int32 * 4)(*[int(x) for x in adapt[0]])
            opt.w_max = (C.c_int32 * 4)(*[int(x) for x in adapt[1]])
        stats = (LsStats * self.n_units)()
        check(lib().mdvrp_local_search_to_optimum(self.handle, C.byref(opt), stats, _stream()))
        return [dict(passes=s.passes, steps=s.steps, moves_applied=s.moves_applied, evaluated=s.evaluated, F=s.F,
                     fallback_passes=s.fallback_passes, device_ms=s.device_ms, converged=s.converged, err=s.err,
                     w_final=[int(x) for x in s.w_final])
                for s in stats]

    # ------------------------------------------------------------------ population (Section 3.4)
    def population_distance(self, units):
        """Eq. 7 between the current solutions of the listed units: device (dist [n][n] fp64,
        common arcs [n][n] int64, |E| [n] int64)."""
        torch = _torch()
        ul = np.ascontiguousarray(units, dtype=np.int32)
        n = len(ul)
        nbytes = C.c_size_t(0)
        check(lib().mdvrp_population_workspace_query(self.handle, ul.ctypes.data_as(C.c_void_p), n,
                                                     C.byref(nbytes)))
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        dist = torch.empty((n, n), dtype=torch.float64, device="cuda")
        common = torch.empty((n, n), dtype=torch.int64, device="cuda")
        ne = torch.empty(n, dtype=torch.int64, device="cuda")
        check(lib().mdvrp_population_distance(self.handle, ul.ctypes.data_as(C.c_void_p), n, _dptr(dist),
                                              _dptr(common), _dptr(ne), _dptr(ws), nbytes.value, _stream()))
        return dist, common, ne

    # ------------------------------------------------------------------ autotuner
    def autotune(self, fam_mask=FAM_ALL, reps=3):
        """Pick the fastest tile shape of each family's evaluation; returns threads per block."""
        out = np.zeros(6, np.int32)
        check(lib().mdvrp_autotune(self.handle, fam_mask, reps, out.ctypes.data_as(C.c_void_p), _stream()))
        return [int(x) for x in out]

    def set_tile_shapes(self, threads):
        arr = np.ascontiguousarray(threads, dtype=np.int32)
        check(lib().mdvrp_set_tile_shapes(self.handle, arr.ctypes.data_as(C.c_void_p)))

    # ------------------------------------------------------------------ learned filter
    def filter_attach(self, k):
        torch = _torch()
        nbytes = C.c_size_t(0)
        check(lib().mdvrp_filter_workspace_query(self.handle, k, C.byref(nbytes)))
        self.filter_ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        check(lib().mdvrp_filter_attach(self.handle, k, _dptr(self.filter_ws), nbytes.value, _stream()))
        self.kc = k

    def anchor_count(self):
        n = C.c_int64(0)
        check(lib().mdvrp_filter_anchor_count(self.handle, C.byref(n)))
        return n.value

    def features(self, as_numpy=True):
        """bf16 bits of every anchor's features, [anchors][32]."""
        torch = _torch()
        out = torch.empty((self.anchor_count(), 32), dtype=torch.int16, device="cuda")
        check(lib().mdvrp_filter_features(self.handle, _dptr(out), _stream()))
        if not as_numpy:
            return out
        torch.cuda.synchronize()
        return out.cpu().numpy().view(np.uint16)

    def labels(self, fam_mask=PAIR_FAMILIES, as_numpy=True):
        torch = _torch()
        out = torch.zeros(self.anchor_count(), dtype=torch.uint8, device="cuda")
        check(lib().mdvrp_filter_labels(self.handle, fam_mask, _dptr(out), _stream()))
        if not as_numpy:
            return out
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def score_topk(self, mlp, want_logits=True):
        torch = _torch()
        lg = torch.full((self.anchor_count(),), float("nan"), dtype=torch.float32, device="cuda") if want_logits else None
        check(lib().mdvrp_filter_score_topk(self.handle, mlp.handle, _dptr(lg) if lg is not None else None, _stream()))
        if lg is None:
            return None
        torch.cuda.synchronize()
        return lg.cpu().numpy()

    def eta_lists(self):
        check(lib().mdvrp_filter_eta_lists(self.handle, _stream()))

    def filter_lists(self):
        """Candidate lists per unit: list of [n_customers][k] arrays."""
        torch = _torch()
        out = torch.empty(int(self.nc.sum()) * self.kc, dtype=torch.int32, device="cuda")
        check(lib().mdvrp_filter_export(self.handle, _dptr(out), _stream()))
        torch.cuda.synchronize()
        a = out.cpu().numpy()
        res, at = [], 0
        for n in self.nc:
            res.append(a[at:at + n * self.kc].reshape(n, self.kc).copy())
            at += n * self.kc
        return res


class Mlp:
    """Scoring network (32 -> 256 -> 256 -> 1) with fp32 master weights and Adam state on the device."""

    def __init__(self, params=None):
        torch = _torch()
        nbytes = C.c_size_t(0)
        check(lib().mdvrp_mlp_workspace_query(C.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        init = None
        if params is not None:
            init = torch.as_tensor(np.ascontiguousarray(params, np.float32)).to("cuda")
        h = C.c_void_p()
        check(lib().mdvrp_mlp_create(_dptr(self.ws), nbytes.value, _dptr(init) if init is not None else None,
                                     _stream(), C.byref(h)))
        self.handle = h
        torch.cuda.synchronize()
        self._act = None
        self._act_n = -1

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mdvrp_mlp_destroy(h)
            self.handle = None

    def get_params(self):
        """Host copy of the fp32 master parameters."""
        torch = _torch()
        p = C.c_void_p()
        check(lib().mdvrp_mlp_params(self.handle, C.byref(p)))
        off = p.value - self.ws.data_ptr()
        torch.cuda.synchronize()
        return self.ws[off:off + 4 * MLP_PARAMS].view(torch.float32).cpu().numpy().copy()

    def set_params(self, params, reset_adam=True):
        torch = _torch()
        p = C.c_void_p()
        check(lib().mdvrp_mlp_params(self.handle, C.byref(p)))
        off = p.value - self.ws.data_ptr()
        src = torch.as_tensor(np.ascontiguousarray(params, np.float32)).to("cuda")
        self.ws[off:off + 4 * MLP_PARAMS].view(torch.float32).copy_(src)
        check(lib().mdvrp_mlp_sync(self.handle, 1 if reset_adam else 0, _stream()))

    def act(self, n):
        torch = _torch()
        if self._act is None or self._act_n < n:
            b = C.c_size_t(0)
            check(lib().mdvrp_mlp_act_bytes(n, C.byref(b)))
            self._act = torch.empty(b.value, dtype=torch.uint8, device="cuda")
            self._act_n = n
            self._act_bytes = b.value
        return self._act, self._act_bytes

    def forward(self, x, keep=False):
        """x: device int16 tensor [n][32] of bf16 bits; returns device fp32 logits."""
        torch = _torch()
        n = x.shape[0]
        z = torch.empty(n, dtype=torch.float32, device="cuda")
        if keep:
            a, ab = self.act(n)
            check(lib().mdvrp_mlp_forward(self.handle, _dptr(x), n, _dptr(z), _dptr(a), ab, _stream()))
        else:
            check(lib().mdvrp_mlp_forward(self.handle, _dptr(x), n, _dptr(z), None, 0, _stream()))
        return z

    def backward(self, x, dz):
        """Gradient of sum dz * logit after forward(x, keep=True); device fp32 [MLP_PARAMS]."""
        torch = _torch()
        n = x.shape[0]
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        a, ab = self.act(n)
        check(lib().mdvrp_mlp_backward(self.handle, _dptr(x), _dptr(dz), n, _dptr(g), _dptr(a), ab, _stream()))
        return g

    def bce(self, z, y, w=None):
        torch = _torch()
        n = z.shape[0]
        dz = torch.empty(n, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        check(lib().mdvrp_mlp_bce(self.handle, _dptr(z), _dptr(y), _dptr(w) if w is not None else None, n, _dptr(dz),
                                  _dptr(loss), _stream()))
        return dz, loss

    def adam(self, g, lr, step):
        check(lib().mdvrp_adam_step(self.handle, _dptr(g), float(lr), int(step), _stream()))

    def train_step(self, x, y, w, lr, step):
        """One optimiser step on (x, y[, w]); returns device (logits, loss, grads)."""
        torch = _torch()
        n = x.shape[0]
        a, ab = self.act(n)
        z = torch.empty(n, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        check(lib().mdvrp_mlp_train_step(self.handle, _dptr(x), _dptr(y), _dptr(w) if w is not None else None, n,
                                         float(lr), int(step), _dptr(g), _dptr(z), _dptr(loss), _dptr(a), ab,
                                         _stream()))
        return z, loss, g

    def train_step_static(self, x, y, w, lr, step):
        """train_step through the allocation-free entry point (n <= TRAIN_STATIC_MAX_N)."""
        torch = _torch()
        n = x.shape[0]
        z = torch.empty(n, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        check(lib().mdvrp_mlp_train_step_static(self.handle, _dptr(x), _dptr(y), _dptr(w) if w is not None else None,
                                                n, float(lr), int(step), _dptr(g), _dptr(z), _dptr(loss),
                                                _stream()))
        return z, loss, g


def population_reduce(dist, f, mu, xi=0.7, n_close=5):
    """Reduce a population to mu members by the score of Eq. 5 (device tensors in, device out):
    (keep [n] int32, removal order [n - mu] int32, chi [n] fp64, population distance [n] fp64)."""
    torch = _torch()
    n = int(f.shape[0])
    keep = torch.empty(n, dtype=torch.int32, device="cuda")
    order = torch.empty(max(n - mu, 1), dtype=torch.int32, device="cuda")
    chi = torch.empty(n, dtype=torch.float64, device="cuda")
    dpop = torch.empty(n, dtype=torch.float64, device="cuda")
    check(lib().mdvrp_population_reduce(_dptr(dist), _dptr(f), n, int(mu), float(xi), int(n_close), _dptr(keep),
                                        _dptr(order), _dptr(chi), _dptr(dpop), _stream()))
    return keep, order[:max(n - mu, 0)], chi, dpop


def _routes_dev(routes):
    nodes, offs, st, en = [], [0], [], []
    for a, xs, b in routes:
        nodes.extend(xs)
        offs.append(len(nodes))
        st.append(a)
        en.append(b)
    pad = lambda v: v if len(v) else [0]  # noqa: E731
    return ([_dev_i32(np.asarray(pad(v), np.int32)) for v in (nodes, offs, st, en)], len(routes), len(nodes))


def dcrex_counts(n_depots, n_nodes, offspring, intro, parent):
    """Route-pair counts of the crossover (Algorithm 3) on the device: (EI, NR, NM, NC) as
    device int32 tensors [ns][np]; offspring / parent are lists of (start, customers, end)."""
    torch = _torch()
    (sn, so, ss, se), ns, s_len = _routes_dev(offspring)
    (pn, po, ps, pe), np_, p_len = _routes_dev(parent)
    it = _dev_i32(np.asarray(intro if len(intro) else [0], np.int32))
    out = [torch.zeros(max(ns * np_, 1), dtype=torch.int32, device="cuda") for _ in range(4)]
    nbytes = C.c_size_t(0)
    check(lib().mdvrp_dcrex_workspace_query(n_nodes, ns, np_, p_len, C.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
    check(lib().mdvrp_dcrex_counts(n_depots, n_nodes, ns, s_len, _dptr(sn), _dptr(so), _dptr(ss), _dptr(se),
                                   _dptr(it), np_, p_len, _dptr(pn), _dptr(po), _dptr(ps), _dptr(pe),
                                   *[_dptr(o) for o in out], _dptr(ws), nbytes.value, _stream()))
    return [o[:ns * np_].reshape(ns, np_) for o in out]


def dcrex_pick(counts, seed):
    """Algorithm 3's exchange among the five lowest pairs: (i, j, diversity increase, candidates)."""
    torch = _torch()
    ei, nr, nm, nc = counts
    ns, np_ = ei.shape
    out = torch.empty(4, dtype=torch.int32, device="cuda")
    check(lib().mdvrp_dcrex_pick(ns, np_, _dptr(ei), _dptr(nr), _dptr(nm), _dptr(nc), int(seed), _dptr(out),
                                 _stream()))
    return [int(v) for v in out.cpu().numpy()]


def ucb_select(R, N):
    """Arm chosen by discounted UCB1 (Eq. 4) from device fp64 tensors R, N."""
    torch = _torch()
    arm = torch.empty(1, dtype=torch.int32, device="cuda")
    check(lib().mdvrp_ucb_select(int(R.shape[0]), _dptr(R), _dptr(N), _dptr(arm), _stream()))
    return arm


def ucb_update(R, N, arm, reward, gamma=0.99):
    """In place on device fp64 tensors R, N; arm a device int32 tensor [1], reward a device fp64 [1]."""
    check(lib().mdvrp_ucb_update(int(R.shape[0]), _dptr(R), _dptr(N), _dptr(arm), _dptr(reward), float(gamma),
                                 _stream()))


def validate_solutions_host(instances, unit_inst, solutions):
    """Host-only validation of solutions (no GPU needed); returns the status."""
    from .gen import batch_flat
    descs = (InstanceDesc * len(instances))(*[desc_from_host(i) for i in instances])
    ui = np.ascontiguousarray(unit_inst, dtype=np.int32)
    nodes, offs, st, en, so = batch_flat(solutions)
    if len(nodes) == 0:
        nodes = np.zeros(1, np.int32)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    return lib().mdvrp_validate_solutions_host(descs, len(instances), ptr(ui), len(ui), ptr(nodes), ptr(offs),
                                               ptr(st), ptr(en), ptr(so))


def validate_instance_host(inst):
    d = desc_from_host(inst)
    return lib().mdvrp_validate_instance_host(C.byref(d))


def family_order(has_tw, seed, p):
    fam = np.zeros(6, np.int32)
    n = lib().mdvrp_family_order(has_tw, seed, p, fam.ctypes.data_as(C.c_void_p))
    return [int(x) for x in fam[:n]]
