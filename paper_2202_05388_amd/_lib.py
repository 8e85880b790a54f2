"""ctypes binding of libgfo (include/gfo.h).  Argument marshalling only.

Every function here forwards to the C ABI of the same name; all arithmetic of
the optimiser runs in the library's HIP kernels.  Loading fails loudly when
the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfo.so")

GFO_C64, GFO_C128 = 0, 1
GFO_FP32, GFO_BF16 = 0, 1
GFO_OK, GFO_EINVAL, GFO_EHIP, GFO_ENOSPC, GFO_ERANGE, GFO_ESCRATCH = 0, -1, -2, -3, -4, -5
GFO_STATUS_SINGULAR, GFO_STATUS_NONFINITE = 1, 2
GFO_STATUS_HISTORY_FULL, GFO_STATUS_REFRESH_OVERFLOW = 4, 8
GFO_MAX_EPS = 8
GFO_MAX_RANK_K = 32
GFO_MAX_DELAY = 128
GFO_STATIC_SCRATCH_BYTES = 8 << 20

# every entry point that include/gfo.h declares
EXPORTS = ("gfo_version", "gfo_strerror", "gfo_last_hip_error", "gfo_workspace_size", "gfo_min_ld", "gfo_g_elems", "gfo_scores_offset",
           "init_G0", "score_candidates", "apply_flip", "apply_flips_rank_k", "refresh_G",
           "gfo_k1_variant_count", "gfo_k1_variant_name", "gfo_k1_set_variant",
           "gfo_k1_get_variant", "gfo_time_next_k1", "gfo_flush", "gfo_flush_variant_count",
           "gfo_flush_variant_name", "gfo_flush_set_variant", "gfo_flush_get_variant",
           "gfo_loop_set_form", "gfo_loop_get_form",
           "gfo_greedy_steps", "gfo_choose_eps_greedy", "score_regions", "gfo_region_pixels",
           "gfo_sync_lower", "score_candidates_static", "gfo_rk_variant_count",
           "gfo_rk_variant_name", "gfo_rk_set_variant", "gfo_rk_get_variant",
           "gfo_job_table_bytes", "gfo_job_table_build", "gfo_greedy_steps_table")


class Problem(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("n_mon", C.c_int32), ("dtype", C.c_int32),
                ("wavelength", C.c_double), ("pitch", C.c_double), ("eps_bg", C.c_double),
                ("h_mon_xy", C.POINTER(C.c_double)), ("fom_monitor", C.c_int32),
                ("n_eps", C.c_int32), ("h_eps_table", C.POINTER(C.c_double))]


class State(C.Structure):
    _fields_ = [("G", C.c_void_p), ("ldG", C.c_int64), ("E", C.c_void_p),
                ("diag64", C.c_void_p), ("eps_idx", C.c_void_p), ("flips", C.c_void_p),
                ("flip_cap", C.c_int32), ("n_flips", C.c_void_p), ("kmax", C.c_int32),
                ("work", C.c_void_p), ("work_bytes", C.c_size_t), ("status", C.c_void_p),
                ("delay", C.c_int32), ("pending_calls", C.c_int32), ("lower_stale", C.c_int32),
                ("packed", C.c_int32)]


class Pick(C.Structure):
    _fields_ = [("pixel", C.c_int32), ("eps_idx", C.c_int32), ("fom_new", C.c_double),
                ("dfom", C.c_double)]


PICK_BYTES = C.sizeof(Pick)
_lib = None


class GfoError(RuntimeError):
    """A libgfo call returned an error; `code` is its GFO_E* value (None when
    the error was found in the binding itself)."""

    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


def lib():
    """Load libgfo.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GfoError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # torch first: its wheel carries its own HIP runtime under the same soname,
    # and libgfo must bind to that one (the runtime that owns torch's device
    # memory and streams).  Loaded first, libgfo would pull in the system copy and
    # torch a second runtime beside it, whose launches then fail.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, S, V = C.POINTER(Problem), C.POINTER(State), C.c_void_p
    L.gfo_version.restype = C.c_char_p
    L.gfo_strerror.restype = C.c_char_p
    L.gfo_strerror.argtypes = [C.c_int]
    L.gfo_last_hip_error.restype = C.c_int32
    L.gfo_last_hip_error.argtypes = [C.POINTER(C.c_char_p)]
    L.gfo_workspace_size.argtypes = [P, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
    L.gfo_min_ld.argtypes = [P]
    L.gfo_min_ld.restype = C.c_int64
    L.gfo_g_elems.argtypes = [P, C.c_int64, C.c_int32, C.POINTER(C.c_int64)]
    L.gfo_scores_offset.argtypes = [P, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
    L.init_G0.argtypes = [P, S, V]
    L.score_candidates.argtypes = [P, S, C.c_uint32, C.c_double, C.c_int32, C.c_int32, V, V]
    L.score_candidates_static.argtypes = [P, S, C.c_uint32, C.c_double, C.c_int32, C.c_int32, V, V]
    L.apply_flip.argtypes = [P, S, V, V]
    L.apply_flips_rank_k.argtypes = [P, S, V, C.c_int32, C.c_int32, V]
    L.refresh_G.argtypes = [P, S, V]
    L.gfo_flush.argtypes = [P, S, V]
    L.gfo_sync_lower.argtypes = [P, S, V]
    L.gfo_greedy_steps.argtypes = [P, S, C.c_int32, C.c_uint32, C.c_double, V, V]
    L.gfo_choose_eps_greedy.argtypes = [V, C.c_int32, C.c_double, C.c_double, C.c_double, V, V]
    L.score_regions.argtypes = [P, S, C.c_int32, C.c_uint32, C.c_double, V, V]
    L.gfo_region_pixels.argtypes = [P, S, C.c_int32, V, V, V]
    L.gfo_job_table_bytes.argtypes = [C.c_int32]
    L.gfo_job_table_bytes.restype = C.c_size_t
    L.gfo_job_table_build.argtypes = [P, S, C.c_int32, C.POINTER(C.c_uint32),
                                      C.POINTER(C.c_double), V, C.c_size_t, V]
    L.gfo_greedy_steps_table.argtypes = [P, S, C.c_int32, C.c_int32, V, V]
    L.gfo_rk_variant_name.argtypes = [C.c_int32]
    L.gfo_rk_variant_name.restype = C.c_char_p
    L.gfo_rk_set_variant.argtypes = [C.c_int32]
    L.gfo_flush_variant_name.argtypes = [C.c_int32]
    L.gfo_flush_variant_name.restype = C.c_char_p
    L.gfo_flush_set_variant.argtypes = [C.c_int32]
    L.gfo_loop_set_form.argtypes = [C.c_int32]
    L.gfo_k1_variant_count.argtypes = [C.c_int32]
    L.gfo_k1_variant_name.argtypes = [C.c_int32, C.c_int32]
    L.gfo_k1_variant_name.restype = C.c_char_p
    L.gfo_k1_set_variant.argtypes = [C.c_int32, C.c_int32]
    L.gfo_k1_get_variant.argtypes = [C.c_int32]
    L.gfo_time_next_k1.argtypes = [C.c_void_p, C.c_void_p]
    _lib = L
    return L


def check(rc: int, what: str) -> None:
    if rc != GFO_OK:
        msg = f"{what} failed: {rc} ({lib().gfo_strerror(rc).decode()})"
        if rc == GFO_EHIP:
            name = C.c_char_p()
            code = lib().gfo_last_hip_error(C.byref(name))
            msg += f" [HIP error {code}: {(name.value or b'').decode()}]"
        raise GfoError(msg, code=rc)


def version() -> str:
    return lib().gfo_version().decode()


def workspace_size(prob: Problem, kmax: int, ld: int = 0) -> int:
    out = C.c_size_t(0)
    check(lib().gfo_workspace_size(C.byref(prob), ld, kmax, C.byref(out)), "gfo_workspace_size")
    return out.value


def scores_offset(prob: Problem, kmax: int, ld: int = 0) -> int:
    out = C.c_size_t(0)
    check(lib().gfo_scores_offset(C.byref(prob), ld, kmax, C.byref(out)), "gfo_scores_offset")
    return out.value


def min_ld(prob: Problem) -> int:
    ld = lib().gfo_min_ld(C.byref(prob))
    if ld < 0:
        raise GfoError("invalid problem")
    return ld


def g_elems(prob: Problem, ld: int = 0, packed: bool = False) -> int:
    """Entries of G for this problem: R x ld dense, or band-packed."""
    out = C.c_int64(0)
    check(lib().gfo_g_elems(C.byref(prob), ld, int(bool(packed)), C.byref(out)), "gfo_g_elems")
    return out.value


def init_G0(prob: Problem, st: State, stream: int) -> None:
    check(lib().init_G0(C.byref(prob), C.byref(st), stream), "init_G0")


def score_candidates(prob, st, cand_mask, tau, topk, min_spacing, d_out, stream) -> None:
    check(lib().score_candidates(C.byref(prob), C.byref(st), cand_mask, tau, topk, min_spacing,
                                 d_out, stream), "score_candidates")


def score_candidates_static(prob, st, cand_mask, tau, topk, min_spacing, d_out, stream) -> None:
    check(lib().score_candidates_static(C.byref(prob), C.byref(st), cand_mask, tau, topk,
                                        min_spacing, d_out, stream), "score_candidates_static")


def apply_flip(prob, st, d_pick, stream) -> None:
    check(lib().apply_flip(C.byref(prob), C.byref(st), d_pick, stream), "apply_flip")


def apply_flips_rank_k(prob, st, d_picks, k, gemm_precision, stream) -> None:
    check(lib().apply_flips_rank_k(C.byref(prob), C.byref(st), d_picks, k, gemm_precision, stream),
          "apply_flips_rank_k")


def refresh_G(prob, st, stream) -> None:
    check(lib().refresh_G(C.byref(prob), C.byref(st), stream), "refresh_G")


def flush(prob, st, stream) -> None:
    check(lib().gfo_flush(C.byref(prob), C.byref(st), stream), "gfo_flush")


def sync_lower(prob, st, stream) -> None:
    check(lib().gfo_sync_lower(C.byref(prob), C.byref(st), stream), "gfo_sync_lower")


def score_regions(prob, st, region, cand_mask, tau, d_out, stream) -> None:
    check(lib().score_regions(C.byref(prob), C.byref(st), region, cand_mask, tau, d_out, stream),
          "score_regions")


def region_pixels(prob, st, region, d_region, d_pixels, stream) -> None:
    check(lib().gfo_region_pixels(C.byref(prob), C.byref(st), region, d_region, d_pixels, stream),
          "gfo_region_pixels")


def choose_eps_greedy(d_top, k, eps, u_explore, u_choice, d_out, stream) -> None:
    check(lib().gfo_choose_eps_greedy(d_top, k, eps, u_explore, u_choice, d_out, stream),
          "gfo_choose_eps_greedy")


def greedy_steps(prob, st, n_steps, cand_mask, tau, d_picks, stream) -> None:
    check(lib().gfo_greedy_steps(C.byref(prob), C.byref(st), n_steps, cand_mask, tau, d_picks,
                                 stream), "gfo_greedy_steps")


def k1_variants(dtype: int):
    L = lib()
    return [L.gfo_k1_variant_name(dtype, i).decode() for i in range(L.gfo_k1_variant_count(dtype))]


def k1_set_variant(dtype: int, idx: int) -> None:
    check(lib().gfo_k1_set_variant(dtype, idx), "gfo_k1_set_variant")


def k1_get_variant(dtype: int) -> int:
    return lib().gfo_k1_get_variant(dtype)


def time_next_k1(before: int, after: int) -> None:
    check(lib().gfo_time_next_k1(before, after), "gfo_time_next_k1")


def job_table_bytes(n_jobs: int) -> int:
    return lib().gfo_job_table_bytes(n_jobs)


def job_table_build(probs, states, masks, taus, d_table, table_bytes, stream) -> None:
    """probs, states: ctypes arrays (Problem * n, State * n); masks, taus: sequences."""
    n = len(probs)
    m = (C.c_uint32 * n)(*[int(x) for x in masks])
    t = (C.c_double * n)(*[float(x) for x in taus])
    check(lib().gfo_job_table_build(probs, states, n, m, t, d_table, table_bytes, stream),
          "gfo_job_table_build")


def greedy_steps_table(probs, states, n_steps, d_table, stream) -> None:
    check(lib().gfo_greedy_steps_table(probs, states, len(probs), n_steps, d_table, stream),
          "gfo_greedy_steps_table")


def rk_variants():
    L = lib()
    return [L.gfo_rk_variant_name(i).decode() for i in range(L.gfo_rk_variant_count())]


def rk_set_variant(idx: int) -> None:
    check(lib().gfo_rk_set_variant(idx), "gfo_rk_set_variant")


def rk_get_variant() -> int:
    return lib().gfo_rk_get_variant()


def flush_variants():
    L = lib()
    return [L.gfo_flush_variant_name(i).decode() for i in range(L.gfo_flush_variant_count())]


def flush_set_variant(idx: int) -> None:
    check(lib().gfo_flush_set_variant(idx), "gfo_flush_set_variant")


def flush_get_variant() -> int:
    return lib().gfo_flush_get_variant()


def loop_set_form(form: int) -> None:
    """Deferred-mode greedy loop: 0 automatic (one kernel per move where the grid
    allows), 1 two kernels per move."""
    check(lib().gfo_loop_set_form(form), "gfo_loop_set_form")


def loop_get_form() -> int:
    return lib().gfo_loop_get_form()
