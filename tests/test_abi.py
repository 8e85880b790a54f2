"""C-ABI checks that need no GPU: the library loads, exports every entry point that
include/gfo.h declares, and rejects invalid arguments on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2202_05388_amd import _lib as L
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    """Names of every function prototype in include/gfo.h (comments stripped)."""
    src = open(os.path.join(ROOT, "include", "gfo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][A-Za-z0-9_]*)\s*\(",
                                 src, flags=re.M)))


def _problem(p, dtype=L.GFO_C128):
    mon = np.ascontiguousarray(p.monitor_xy().reshape(-1))
    eps = np.ascontiguousarray(p.eps_table, dtype=np.float64)
    pr = L.Problem(ny=p.ny, nx=p.nx, n_mon=p.n_mon, dtype=dtype, wavelength=p.wavelength,
                   pitch=p.pitch, eps_bg=1.0, h_mon_xy=mon.ctypes.data_as(C.POINTER(C.c_double)),
                   fom_monitor=p.fom_monitor, n_eps=len(eps),
                   h_eps_table=eps.ctypes.data_as(C.POINTER(C.c_double)))
    return pr, (mon, eps)


def test_library_exports_every_declared_entry_point():
    lib = L.lib()
    declared = _declared_functions()
    for name in ("init_G0", "score_candidates", "apply_flip", "apply_flips_rank_k", "refresh_G",
                 "gfo_workspace_size", "gfo_strerror", "gfo_version", "gfo_flush", "gfo_time_next_k1"):
        assert name in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) <= set(L.EXPORTS)
    assert "gfx950" in L.version()


def test_struct_layouts_match_header():
    # x86-64 SysV layout of the structs in include/gfo.h
    assert C.sizeof(L.Problem) == 64
    assert L.Problem.h_mon_xy.offset == 40 and L.Problem.h_eps_table.offset == 56
    assert C.sizeof(L.State) == 112
    assert L.State.work.offset == 72 and L.State.status.offset == 88
    assert L.State.delay.offset == 96 and L.State.pending_calls.offset == 100
    assert L.State.lower_stale.offset == 104 and L.State.packed.offset == 108
    assert C.sizeof(L.Pick) == 24


def test_workspace_size_and_leading_dimension():
    pr, keep = _problem(W.SQUARE_128)
    assert L.min_ld(pr) == 16384
    small = L.workspace_size(pr, 0)
    big = L.workspace_size(pr, 256)
    R = 16384 + 64
    assert big - small >= 2 * R * 256 * 16       # U and Z refresh panels
    pr2, keep2 = _problem(W.tiny(5, 7, n_mon=3))
    assert L.min_ld(pr2) == 64
    assert L.scores_offset(pr2, 0) % 256 == 0
    # a padded leading dimension grows the workspace; invalid ones are refused
    assert L.workspace_size(pr, 0, 16384 + 64) > small
    out = C.c_size_t(0)
    for bad in (16384 - 64, 16384 + 32):
        assert L.lib().gfo_workspace_size(C.byref(pr), bad, 0, C.byref(out)) == L.GFO_EINVAL


@pytest.mark.parametrize("field,value", [("ny", 0), ("n_mon", 0), ("dtype", 7), ("wavelength", 0.0),
                                         ("fom_monitor", 99), ("n_eps", 1), ("n_eps", 9)])
def test_invalid_problem_rejected_on_host(field, value):
    pr, keep = _problem(W.tiny(4, 4))
    setattr(pr, field, value)
    out = C.c_size_t(0)
    assert L.lib().gfo_workspace_size(C.byref(pr), 0, 0, C.byref(out)) == L.GFO_EINVAL
    st = L.State()
    assert L.lib().init_G0(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL


def test_background_must_be_in_table():
    p = W.tiny(4, 4).replace(eps_table=(2.0, 12.25))
    pr, keep = _problem(p)
    assert L.lib().gfo_min_ld(C.byref(pr)) == -1


def test_null_state_and_bad_ld_rejected_without_gpu_work():
    pr, keep = _problem(W.tiny(4, 4))
    st = L.State()     # all null
    lib = L.lib()
    assert lib.init_G0(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL
    assert lib.score_candidates(C.byref(pr), C.byref(st), 3, 1e-9, 1, 0, None, None) == L.GFO_EINVAL
    assert lib.apply_flip(C.byref(pr), C.byref(st), None, None) == L.GFO_EINVAL
    assert lib.apply_flips_rank_k(C.byref(pr), C.byref(st), None, 4, 0, None) == L.GFO_EINVAL
    assert lib.refresh_G(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL
    assert lib.gfo_flush(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL
    # non-null but fake pointers with a bad leading dimension: rejected before any launch
    fake = 1 << 20
    st = L.State(G=fake, ldG=17, E=fake, diag64=fake, eps_idx=fake, flips=fake, flip_cap=4,
                 n_flips=fake, kmax=0, work=fake, work_bytes=1 << 30, status=fake)
    assert lib.init_G0(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL
    st.ldG = 64
    st.delay = 129                              # above GFO_MAX_DELAY
    assert lib.init_G0(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL
    st.delay = 0
    st.work_bytes = 16
    assert lib.init_G0(C.byref(pr), C.byref(st), None) == L.GFO_ENOSPC


def test_k1_variants_listed():
    for dt in (L.GFO_C64, L.GFO_C128):
        names = L.k1_variants(dt)
        assert len(names) >= 4 and len(set(names)) == len(names)
    assert L.lib().gfo_k1_set_variant(L.GFO_C64, 999) == L.GFO_EINVAL
    assert L.flush_variants() == ["w32_3m", "up_pair4_3m_nt", "up_pair4_3m_nt_x8", "up_band4_3m_nt",
                                  "up_bandseg4_3m_nt", "up_bandseg_s3"]
    assert L.flush_get_variant() == 5
    assert L.rk_variants()[0] == "acc64" and len(set(L.rk_variants())) == len(L.rk_variants())
    assert L.lib().gfo_strerror(L.GFO_ENOSPC) == b"workspace too small"
    # no HIP call of the library has failed on this thread
    assert L.lib().gfo_last_hip_error(None) == 0


def test_choose_eps_greedy_rejects_bad_arguments_on_host():
    lib = L.lib()
    fake = C.c_void_p(256)          # never dereferenced: every case fails validation first
    for k, eps, u1, u2 in ((0, 0.1, 0.5, 0.5), (33, 0.1, 0.5, 0.5), (4, -0.1, 0.5, 0.5),
                           (4, 1.5, 0.5, 0.5), (4, 0.1, 1.0, 0.5), (4, 0.1, 0.5, -0.2)):
        assert lib.gfo_choose_eps_greedy(fake, k, eps, u1, u2, fake, None) == L.GFO_EINVAL
    assert lib.gfo_choose_eps_greedy(None, 4, 0.1, 0.5, 0.5, fake, None) == L.GFO_EINVAL


def test_region_calls_reject_bad_region_on_host():
    """Another region side, or an odd grid, is refused before anything is launched."""
    lib = L.lib()
    pr, keep = _problem(W.tiny(8, 8, n_mon=4))
    ld = L.min_ld(pr)
    work = L.workspace_size(pr, 0)
    fake = 1 << 20                       # aligned, never dereferenced
    st = L.State(G=fake, ldG=ld, E=fake, diag64=fake, eps_idx=fake, flips=fake, flip_cap=16,
                 n_flips=fake, kmax=0, work=fake, work_bytes=work, status=fake, delay=0,
                 pending_calls=0)
    out = C.c_void_p(fake)
    for region in (0, 1, 3, 4):
        assert lib.score_regions(C.byref(pr), C.byref(st), region, 3, 1e-9, out, None) == L.GFO_EINVAL
        assert lib.gfo_region_pixels(C.byref(pr), C.byref(st), region, out, out, None) == L.GFO_EINVAL
    pr2, keep2 = _problem(W.tiny(7, 8, n_mon=4))
    st2 = L.State(G=fake, ldG=L.min_ld(pr2), E=fake, diag64=fake, eps_idx=fake, flips=fake,
                  flip_cap=16, n_flips=fake, kmax=0, work=fake, work_bytes=L.workspace_size(pr2, 0),
                  status=fake, delay=0, pending_calls=0)
    assert lib.score_regions(C.byref(pr2), C.byref(st2), 2, 3, 1e-9, out, None) == L.GFO_EINVAL


def test_sync_lower_validates_and_is_a_no_op_when_current():
    """gfo_sync_lower refuses a flag other than 0 or 1 and launches nothing when
    the lower triangle is current (the pointers here are never dereferenced)."""
    lib = L.lib()
    pr, keep = _problem(W.tiny(8, 8, n_mon=4))
    fake = 1 << 20
    st = L.State(G=fake, ldG=L.min_ld(pr), E=fake, diag64=fake, eps_idx=fake, flips=fake,
                 flip_cap=16, n_flips=fake, kmax=0, work=fake, work_bytes=L.workspace_size(pr, 0),
                 status=fake, delay=16, pending_calls=0, lower_stale=0)
    assert lib.gfo_sync_lower(C.byref(pr), C.byref(st), None) == L.GFO_OK
    st.lower_stale = 2
    assert lib.gfo_sync_lower(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL
    assert lib.gfo_flush(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL


def test_loop_form_hook_validates_and_round_trips():
    """gfo_loop_set_form accepts 0 (automatic) and 1 (two kernels per move) only;
    host-side state, no device work."""
    lib = L.lib()
    old = L.loop_get_form()
    assert old == 0
    try:
        assert lib.gfo_loop_set_form(2) == L.GFO_EINVAL
        assert lib.gfo_loop_set_form(-1) == L.GFO_EINVAL
        assert L.loop_get_form() == old
        L.loop_set_form(1)
        assert L.loop_get_form() == 1
    finally:
        L.loop_set_form(old)
    assert L.loop_get_form() == 0


def test_static_score_rejects_oversize_and_bad_arguments_on_host():
    """score_candidates_static refuses a problem whose scores would not fit its
    8 MiB device scratch (GFO_ESCRATCH) and invalid arguments (GFO_EINVAL),
    before any HIP call; it needs no workspace (work may be NULL)."""
    lib = L.lib()
    fake = 1 << 20                                 # aligned, never dereferenced
    out = C.c_void_p(fake)

    def state(pr):
        return L.State(G=fake, ldG=L.min_ld(pr), E=fake, diag64=fake, eps_idx=fake, flips=fake,
                       flip_cap=16, n_flips=fake, kmax=0, work=None, work_bytes=0, status=fake)

    # 1024 x 1024 pixels with two materials: 16 MiB of scores
    big, keep = _problem(W.tiny(1024, 1024, n_mon=4))
    st = state(big)
    assert lib.score_candidates_static(C.byref(big), C.byref(st), 3, 1e-9, 1, 0, out,
                                       None) == L.GFO_ESCRATCH
    assert lib.gfo_strerror(L.GFO_ESCRATCH) == b"problem too large for the library's static scratch"
    # the largest grid that fits: N * n_eps * 8 bytes + 12 KiB of summaries <= 8 MiB
    assert (L.GFO_STATIC_SCRATCH_BYTES - 12288) // 16 == 523_520
    small, keep2 = _problem(W.tiny(8, 8, n_mon=4))
    st = state(small)
    for mask, tau, topk, spacing in ((0, 1e-9, 1, 0), (3, -1.0, 1, 0), (3, 1e-9, 0, 0),
                                     (3, 1e-9, 33, 0), (3, 1e-9, 4, -1)):
        assert lib.score_candidates_static(C.byref(small), C.byref(st), mask, tau, topk, spacing,
                                           out, None) == L.GFO_EINVAL
    assert lib.score_candidates_static(C.byref(small), C.byref(st), 3, 1e-9, 1, 0, None,
                                       None) == L.GFO_EINVAL
    st.G = None
    assert lib.score_candidates_static(C.byref(small), C.byref(st), 3, 1e-9, 1, 0, out,
                                       None) == L.GFO_EINVAL


def test_packed_storage_sizes_and_refusals():
    """Band-packed G: the entry count (the design bands on and above the
    diagonal, then the monitor rows), and the calls that refuse it before any
    launch: eager updates (delay 0), the rank-k update and gfo_sync_lower (the
    pointers here are never dereferenced)."""
    lib = L.lib()
    for ny, nx, nmon, pad in ((128, 128, 64, 0), (60, 62, 20, 64), (1, 3, 1, 0), (8, 8, 70, 0)):
        pr, keep = _problem(W.tiny(ny, nx, n_mon=nmon))
        N, R = ny * nx, ny * nx + nmon
        ld = L.min_ld(pr) + pad
        assert L.g_elems(pr, ld, False) == R * ld
        # band b holds 64 rows of ld - 64 b entries (the last band's rows past N too)
        nb = (N + 63) // 64
        want = sum(64 * (ld - 64 * b) for b in range(nb)) + nmon * ld
        assert L.g_elems(pr, ld, True) == want
        assert L.g_elems(pr, ld, True) < R * ld or N <= 64
    pr, keep = _problem(W.SQUARE_128, dtype=L.GFO_C64)
    assert L.g_elems(pr, 0, True) * 8 / 1e9 < 0.55 * L.g_elems(pr, 0, False) * 8 / 1e9
    out = C.c_int64(0)
    assert lib.gfo_g_elems(C.byref(pr), 0, 2, C.byref(out)) == L.GFO_EINVAL
    assert lib.gfo_g_elems(C.byref(pr), 17, 1, C.byref(out)) == L.GFO_EINVAL
    pr, keep = _problem(W.tiny(8, 8, n_mon=4), dtype=L.GFO_C64)
    ld = L.min_ld(pr)
    fake = 1 << 20
    st = L.State(G=fake, ldG=ld, E=fake, diag64=fake, eps_idx=fake, flips=fake, flip_cap=16,
                 n_flips=fake, kmax=0, work=fake, work_bytes=L.workspace_size(pr, 0), status=fake,
                 delay=0, pending_calls=0, lower_stale=0, packed=1)
    picks = C.c_void_p(fake)
    # packed needs deferred updates: every call validates that
    assert lib.init_G0(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL
    assert lib.apply_flip(C.byref(pr), C.byref(st), picks, None) == L.GFO_EINVAL
    assert lib.gfo_greedy_steps(C.byref(pr), C.byref(st), 4, 3, 1e-6, None, None) == L.GFO_EINVAL
    st.packed = 2
    st.delay = 16
    assert lib.init_G0(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL
    st.packed = 1
    assert lib.apply_flips_rank_k(C.byref(pr), C.byref(st), picks, 4, L.GFO_FP32, None) == L.GFO_EINVAL
    assert lib.gfo_sync_lower(C.byref(pr), C.byref(st), None) == L.GFO_EINVAL


def test_one_hip_runtime_when_the_library_loads_first():
    """Loaded before torch is imported, libgfo still binds to the HIP runtime of
    torch's wheel: the process maps one libamdhip64."""
    import subprocess
    import sys
    script = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2202_05388_amd import _lib as L\n"
        "L.lib()\n"
        "import torch\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"
