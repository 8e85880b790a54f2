"""One optimisation job: device buffers (torch allocations) + calls into libgfo.

PyTorch provides device memory and the stream; every computation is a libgfo
call.  A problem is any object with the attributes ny, nx, n_mon, wavelength,
pitch, eps_table, cand_mask, dtype, tau, fom_monitor, monitor_xy() (the shared
workload definitions satisfy this).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

_DTYPES = {"c64": (L.GFO_C64, torch.complex64, 8), "c128": (L.GFO_C128, torch.complex128, 16)}


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Job:
    """Device state of one greedy optimisation."""

    def __init__(self, problem, device="cuda", kmax: int = 0, flip_cap: int = None,
                 dtype: str = None, delay: int = 0, ld_pad: int = 0, upper: bool = False,
                 packed: bool = False):
        if not torch.cuda.is_available():
            raise L.GfoError("libgfo needs a GPU; torch.cuda is not available")
        L.lib()
        self.problem = problem
        self.dtype_name = dtype or problem.dtype
        code, tdtype, esize = _DTYPES[self.dtype_name]
        self.device = torch.device(device)
        self.N = problem.ny * problem.nx
        self.R = self.N + problem.n_mon
        self._mon = np.ascontiguousarray(problem.monitor_xy(), dtype=np.float64).reshape(-1)
        self._eps = np.ascontiguousarray(problem.eps_table, dtype=np.float64)
        self.prob = L.Problem(
            ny=problem.ny, nx=problem.nx, n_mon=problem.n_mon, dtype=code,
            wavelength=float(problem.wavelength), pitch=float(problem.pitch), eps_bg=1.0,
            h_mon_xy=self._mon.ctypes.data_as(C.POINTER(C.c_double)),
            fom_monitor=int(problem.fom_monitor), n_eps=len(self._eps),
            h_eps_table=self._eps.ctypes.data_as(C.POINTER(C.c_double)))
        if ld_pad < 0 or ld_pad % 64:
            raise L.GfoError("ld_pad must be a non-negative multiple of 64")
        self.ld = L.min_ld(self.prob) + int(ld_pad)   # padding breaks power-of-two row strides
        self.kmax = int(kmax)
        self.flip_cap = int(flip_cap if flip_cap is not None else max(4 * self.N, 16))
        work_bytes = L.workspace_size(self.prob, self.kmax, self.ld)
        dev = self.device
        # band-packed storage (the design block's upper triangle and the monitor
        # rows, about half of G) works with deferred updates only
        self.packed = bool(packed)
        if self.packed and int(delay) < 1:
            raise L.GfoError("band-packed storage needs deferred updates (delay >= 1)")
        if self.packed:
            self.G = torch.empty((L.g_elems(self.prob, self.ld, True),), dtype=tdtype, device=dev)
        else:
            self.G = torch.empty((self.R, self.ld), dtype=tdtype, device=dev)
        self.E = torch.empty((self.R,), dtype=tdtype, device=dev)
        self.diag64 = torch.empty((self.N,), dtype=torch.complex128, device=dev)
        self.eps_idx = torch.empty((self.N,), dtype=torch.uint8, device=dev)
        self.flips = torch.zeros((2 * self.flip_cap,), dtype=torch.int32, device=dev)
        self.counters = torch.zeros((4,), dtype=torch.int32, device=dev)   # n_flips, status
        self.work = torch.empty((work_bytes,), dtype=torch.uint8, device=dev)
        self.picks = torch.zeros((L.GFO_MAX_RANK_K * L.PICK_BYTES,), dtype=torch.uint8, device=dev)
        self.state = L.State(
            G=self.G.data_ptr(), ldG=self.ld, E=self.E.data_ptr(), diag64=self.diag64.data_ptr(),
            eps_idx=self.eps_idx.data_ptr(), flips=self.flips.data_ptr(), flip_cap=self.flip_cap,
            n_flips=self.counters.data_ptr(), kmax=self.kmax, work=self.work.data_ptr(),
            work_bytes=work_bytes, status=self.counters.data_ptr() + 4, delay=int(delay),
            pending_calls=0, lower_stale=0, packed=int(self.packed))
        self.delay = int(delay)
        # keep only the upper triangle of the (symmetric) design block current,
        # in eager mode too: init_G0 and refresh_G are called with lower_stale = 1
        self.upper = bool(upper)
        self.steps_issued = 0

    # ------------------------------------------------------------------ C-ABI calls
    def init(self, stream=None):
        if self.upper:
            self.state.lower_stale = 1
        L.init_G0(self.prob, self.state, _stream_handle(stream))

    def score(self, topk=1, min_spacing=0, tau=None, cand_mask=None, out=None, stream=None):
        tau = self.problem.tau if tau is None else tau
        mask = self.problem.cand_mask if cand_mask is None else cand_mask
        ptr = self.picks.data_ptr() if out is None else out
        L.score_candidates(self.prob, self.state, mask, tau, topk, min_spacing, ptr,
                           _stream_handle(stream))

    def apply(self, pick_ptr=None, stream=None):
        ptr = self.picks.data_ptr() if pick_ptr is None else pick_ptr
        L.apply_flip(self.prob, self.state, ptr, _stream_handle(stream))

    def apply_rank_k(self, k, precision=L.GFO_FP32, pick_ptr=None, stream=None):
        ptr = self.picks.data_ptr() if pick_ptr is None else pick_ptr
        L.apply_flips_rank_k(self.prob, self.state, ptr, k, precision, _stream_handle(stream))

    def refresh(self, stream=None):
        if self.upper:
            self.state.lower_stale = 1
        L.refresh_G(self.prob, self.state, _stream_handle(stream))

    def flush(self, stream=None):
        """Deferred mode: bring the design block of G up to date (no-op otherwise);
        its lower triangle may stay out of date (see sync_lower)."""
        L.flush(self.prob, self.state, _stream_handle(stream))

    def sync_lower(self, stream=None):
        """Copy the upper triangle of the design block into the lower one if a
        flush left the lower one out of date (band-packed storage keeps no lower
        triangle: a no-op)."""
        if not self.packed:
            L.sync_lower(self.prob, self.state, _stream_handle(stream))

    def _bands(self):
        """(first row, rows, first column, packed offset, row stride) of each
        64-row band of the design block in band-packed storage, then the monitor
        rows' (N, N_m, 0, offset, ld)."""
        ld, N = self.ld, self.N
        out = []
        for b in range((N + 63) // 64):
            r0 = 64 * b
            out.append((r0, min(64, N - r0), r0, 64 * (b * ld - 32 * b * (b - 1)), ld - r0))
        nb = (N + 63) // 64
        out.append((N, self.R - N, 0, 64 * (nb * ld - 32 * nb * (nb - 1)), ld))
        return out

    def dense_G(self):
        """G as an R x ld device tensor.  Band-packed storage: the stored
        entries in place, the design block's lower triangle from its upper one
        (entries left of a row's band and the stale lower halves of the diagonal
        tiles are not used)."""
        if not self.packed:
            return self.G
        D = torch.zeros((self.R, self.ld), dtype=self.G.dtype, device=self.device)
        for r0, nr, c0, off, stride in self._bands():
            if nr <= 0:
                continue
            blk = self.G[off: off + nr * stride].view(nr, stride)
            D[r0: r0 + nr, c0:] = blk[:, : self.ld - c0]
        N = self.N
        up = torch.triu(D[:N, :N])
        D[:N, :N] = up + torch.triu(up, 1).transpose(0, 1)
        return D

    def step(self, stream=None):
        """One greedy step: score + select + rank-1 apply, no host synchronisation."""
        self.score(stream=stream)
        self.apply(stream=stream)
        self.steps_issued += 1

    def greedy_steps(self, n, tau=None, cand_mask=None, out=None, stream=None):
        """n greedy steps through gfo_greedy_steps (fused kernels in deferred
        mode); `out`: device pointer to n pick records, or None."""
        tau = self.problem.tau if tau is None else tau
        mask = self.problem.cand_mask if cand_mask is None else cand_mask
        L.greedy_steps(self.prob, self.state, n, mask, tau, out, _stream_handle(stream))
        self.steps_issued += n

    def eps_greedy_step(self, eps, u_explore, u_choice, n_top=4, stream=None):
        """One epsilon-greedy step (paper Sec. V): top-n_top scores, the policy's
        choice (records 0..n_top-1 and 8 of the pick buffer), rank-1 apply."""
        base = self.picks.data_ptr()
        chosen = base + 8 * L.PICK_BYTES
        self.score(topk=n_top, min_spacing=0, out=base, stream=stream)
        L.choose_eps_greedy(base, n_top, float(eps), float(u_explore), float(u_choice), chosen,
                            _stream_handle(stream))
        self.apply(pick_ptr=chosen, stream=stream)
        self.steps_issued += 1

    def run_eps_greedy(self, eps, draws, max_steps=None, poll_every=32, fused=True, stream=None):
        """Epsilon-greedy trajectory; step t uses draws[t] = (u_explore, u_choice).
        Polls the move counter every poll_every steps and stops once a step made no
        move (every earlier step moved: the policy only takes improving moves).

        fused: a step whose draw does not explore (u_explore >= eps) takes the
        greedy pick, the first record of the top-n selection, so runs of such
        steps go through gfo_greedy_steps (one kernel per move in deferred mode);
        the exploring steps take the top-4 scores and the drawn choice.  Bit for
        bit the per-step path's moves and state (fused=False: every step through
        eps_greedy_step).
        Returns the number of moves made by this call."""
        start = self.n_flips()
        n = len(draws) if max_steps is None else min(max_steps, len(draws))
        t = 0
        while t < n:
            end = min(t + poll_every, n)
            while t < end:
                if not fused or draws[t][0] < eps:
                    self.eps_greedy_step(eps, draws[t][0], draws[t][1], stream=stream)
                    t += 1
                else:
                    u = t
                    while u < end and not draws[u][0] < eps:
                        u += 1
                    self.greedy_steps(u - t, stream=stream)
                    t = u
            if self.n_flips() - start < t:
                break
        return self.n_flips() - start

    def region_step(self, apply="sequential", log_ptr=None, stream=None):
        """One greedy region move (2x2 pixels, paper Sec. II with N_V = 4):
        score_regions, its pixel moves (records 16..19 of the pick buffer), then
        the rank-1 updates one after the other ("sequential") or the joint rank-k
        step ("rank_k", complex64 storage).  The region pick goes to log_ptr
        (device) or record 12."""
        base = self.picks.data_ptr()
        rpick = base + 12 * L.PICK_BYTES if log_ptr is None else log_ptr
        pix = base + 16 * L.PICK_BYTES
        h = _stream_handle(stream)
        region = self.problem.region if self.problem.region > 1 else 2
        L.score_regions(self.prob, self.state, region, self.problem.cand_mask, self.problem.tau,
                        rpick, h)
        L.region_pixels(self.prob, self.state, region, rpick, pix, h)
        n = region * region
        if apply == "rank_k":
            if self.delay and self.state.pending_calls:
                self.flush(stream)
            L.apply_flips_rank_k(self.prob, self.state, pix, n, L.GFO_FP32, h)
        else:
            for i in range(n):
                self.apply(pick_ptr=pix + i * L.PICK_BYTES, stream=stream)
        self.steps_issued += 1

    def run_region_greedy(self, max_steps, poll_every=32, apply="sequential", refresh_every=0,
                          stream=None):
        """Greedy loop over region moves; each step's region pick is logged on the
        device and read at every poll; the loop stops at the first step that found
        no improving region move (later steps of its chunk are no-ops).  With
        refresh_every > 0, refresh_G runs after every refresh_every region moves.
        Returns (region moves made, their region picks as (region, material))."""
        log = torch.zeros(poll_every * L.PICK_BYTES, dtype=torch.uint8, device=self.device)
        moves = []
        done = 0
        while done < max_steps:
            chunk = min(poll_every, max_steps - done)
            if refresh_every:
                chunk = min(chunk, refresh_every - len(moves) % refresh_every)
            for i in range(chunk):
                self.region_step(apply=apply, log_ptr=log.data_ptr() + i * L.PICK_BYTES,
                                 stream=stream)
            done += chunk
            raw = log[: chunk * L.PICK_BYTES].cpu().numpy().tobytes()
            recs = (L.Pick * chunk).from_buffer_copy(raw)
            made = [(r.pixel, r.eps_idx) for r in recs if r.pixel >= 0]
            moves.extend(made)
            if len(made) < chunk:
                break
            if refresh_every and len(moves) % refresh_every == 0:
                self.refresh(stream)
        return len(moves), moves

    # ------------------------------------------------------------------ host views
    def read_picks(self, k=1):
        raw = self.picks[: k * L.PICK_BYTES].cpu().numpy().tobytes()
        arr = (L.Pick * k).from_buffer_copy(raw)
        return [(p.pixel, p.eps_idx, p.fom_new, p.dfom) for p in arr]

    def n_flips(self) -> int:
        return int(self.counters[0].item())

    def status(self) -> int:
        return int(self.counters[1].item())

    def history(self):
        n = min(self.n_flips(), self.flip_cap)
        return self.flips[: 2 * n].view(-1, 2).cpu().numpy()

    def fom(self) -> float:
        e = self.E[self.N + self.problem.fom_monitor].cpu().to(torch.complex128).item()
        return float(e.real**2 + e.imag**2)

    def scores(self):
        off = L.scores_offset(self.prob, self.kmax, self.ld)
        n = self.N * len(self._eps)
        raw = self.work[off: off + 8 * n]
        return raw.view(torch.float64).cpu().numpy().reshape(self.N, len(self._eps))

    def host_state(self):
        """(G[:, :N], E, diag64, eps_idx) copied to host numpy, complex128 (flushes
        and completes the lower triangle first)."""
        self.flush()
        self.sync_lower()
        torch.cuda.synchronize(self.device)
        G = self.dense_G()[:, : self.N].cpu().to(torch.complex128).numpy()
        return (G, self.E.cpu().to(torch.complex128).numpy(), self.diag64.cpu().numpy(),
                self.eps_idx.cpu().numpy())

    def upload_state(self, G, E, diag, eps_idx):
        """Overwrite the device state with host arrays (tests build arbitrary states this way)."""
        _, tdtype, _ = _DTYPES[self.dtype_name]
        Gt = torch.zeros((self.R, self.ld), dtype=torch.complex128)
        # np.array copies: read-only views (np.diagonal) are not valid tensor storage
        Gt[:, : self.N] = torch.from_numpy(np.array(G, np.complex128))
        if self.packed:
            for r0, nr, c0, off, stride in self._bands():
                if nr > 0:
                    self.G[off: off + nr * stride].view(nr, stride).copy_(
                        Gt[r0: r0 + nr, c0: c0 + stride].to(tdtype))
        else:
            self.G.copy_(Gt.to(tdtype))
        self.E.copy_(torch.from_numpy(np.array(E, np.complex128)).to(tdtype))
        self.diag64.copy_(torch.from_numpy(np.array(diag, np.complex128)))
        self.eps_idx.copy_(torch.from_numpy(np.array(eps_idx, np.uint8)))
        torch.cuda.synchronize(self.device)
        self.state.lower_stale = 0                    # the whole matrix was written

    def set_pick(self, pixel, eps_idx, slot=0):
        rec = L.Pick(pixel=pixel, eps_idx=eps_idx, fom_new=0.0, dfom=0.0)
        raw = torch.frombuffer(bytearray(bytes(rec)), dtype=torch.uint8)
        self.picks[slot * L.PICK_BYTES:(slot + 1) * L.PICK_BYTES].copy_(raw)

    def run_greedy(self, max_steps, poll_every=32, refresh_every=0, stream=None, fused=False):
        """Greedy loop.  Steps are issued without host synchronisation; after
        each chunk of at most `poll_every` steps the accepted-move counter is
        read and the loop stops once a step found no improving move (that step
        and any later ones in its chunk are no-ops on the device).  With
        refresh_every > 0, refresh_G runs whenever the number of moves accepted
        since init_G0 reaches a multiple of refresh_every.  fused: each chunk
        is one gfo_greedy_steps call (same moves and state).
        Returns the number of moves accepted by this call."""
        start = self.n_flips()
        acc = start
        done = 0
        while done < max_steps:
            chunk = min(poll_every, max_steps - done)
            if refresh_every:
                chunk = min(chunk, refresh_every - acc % refresh_every)
            if fused:
                self.greedy_steps(chunk, stream=stream)
            else:
                for _ in range(chunk):
                    self.step(stream)
            done += chunk
            now = self.n_flips()
            stopped = now - acc < chunk
            acc = now
            if stopped:
                break
            if refresh_every and acc % refresh_every == 0:
                self.refresh(stream)
        return acc - start

    # ------------------------------------------------------------------ HIP graphs
    def capture_steps(self, n: int, stream=None, fused=False):
        """Capture n greedy steps (score + select + apply, and in deferred mode the
        flush that ends a window of `delay` steps) into a HIP graph on `stream`;
        fused: as one gfo_greedy_steps call.

        Capture records launches only; nothing runs.  The window must start with
        no pending deferred terms, and n a multiple of delay in deferred mode, so
        that every replay ends with its own flush and leaves no pending term."""
        if self.delay:
            if n % self.delay or self.state.pending_calls:
                raise L.GfoError("graph window must be a multiple of delay and start flushed")
        s = stream if stream is not None else torch.cuda.Stream(device=self.device)
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize(self.device)
        with torch.cuda.graph(g, stream=s):
            if fused:
                self.greedy_steps(n, stream=s)
            else:
                for _ in range(n):
                    self.score(stream=s)
                    self.apply(stream=s)
        return g, s

    def run_greedy_graph(self, max_steps, window=64, refresh_every=0, fused=False):
        """Greedy loop that replays a captured window of steps; polls and refreshes
        between replays.  Returns the number of moves accepted by this call."""
        if refresh_every and refresh_every % window:
            raise L.GfoError("refresh_every must be a multiple of the window")
        g, s = self.capture_steps(window, fused=fused)
        start = self.n_flips()
        acc = start
        done = 0
        while done < max_steps:
            g.replay()
            done += window
            now = self.n_flips()
            stopped = now - acc < window
            acc = now
            if stopped:
                break
            if refresh_every and acc % refresh_every == 0:
                self.refresh()
        return acc - start


class JobGroup:
    """Resident jobs stepped together: one launch per move for all of them
    (gfo_greedy_steps_table) instead of one per job.  Every job must be in
    deferred mode, and the jobs alike in storage type, term batch and grid class
    (the library refuses other groups).  The device job table is rebuilt by
    `build` whenever the set of jobs changes."""

    def __init__(self, jobs, device="cuda"):
        self.device = torch.device(device)
        self.jobs = []
        self.table = None
        self._probs = None
        self.set_jobs(jobs)

    def set_jobs(self, jobs):
        self.jobs = list(jobs)
        self._probs = None
        self.table = None

    def __len__(self):
        return len(self.jobs)

    def build(self, stream=None):
        """Write the device table of the current jobs (synchronises `stream`)."""
        n = len(self.jobs)
        if n == 0:
            self.table = None
            return
        self._probs = (L.Problem * n)(*[j.prob for j in self.jobs])
        nbytes = L.job_table_bytes(n)
        self.table = torch.empty((nbytes,), dtype=torch.uint8, device=self.device)
        states = (L.State * n)(*[j.state for j in self.jobs])
        L.job_table_build(self._probs, states, [j.problem.cand_mask for j in self.jobs],
                          [j.problem.tau for j in self.jobs], self.table.data_ptr(), nbytes,
                          _stream_handle(stream))

    def steps(self, n, stream=None):
        """n greedy moves of every job: per job, bit for bit the results of one
        greedy_steps(n) call."""
        if self.table is None:
            raise L.GfoError("JobGroup.build() must run after the set of jobs changes")
        states = (L.State * len(self.jobs))(*[j.state for j in self.jobs])
        L.greedy_steps_table(self._probs, states, n, self.table.data_ptr(), _stream_handle(stream))
        for j, st in zip(self.jobs, states):
            j.state.pending_calls = st.pending_calls
            j.steps_issued += n
