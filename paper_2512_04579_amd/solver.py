"""Outer loops built from the C-ABI calls: Alg. 1 (GN-MPPI, Methods D and E)
and deterministic MPPI (Method C).

Each iteration only enqueues library calls on the current stream; the step
length, the new cost and every status word stay in device memory, so an
iteration never waits for the GPU and can be captured into a HIP graph.  The
host computes only the scalar sampling scale of the iteration.

Readings of the paper used here: Alg. 1 shrinks the covariance,
Sigma_{k+1} = beta Sigma_k, so the sampler's scale is
sigma_k = max(sigma_0 beta^(k/2), sigma_min); the step-length set is
{gamma^j : j < L}; the GGN step uses the nominal residual R(U_k).
"""
from __future__ import annotations

import torch

from . import _lib
from .problem import DeviceProblem

_ALIGN = 64  # leading dimensions are padded to 64 elements (256 B for float)


def _round_up(v: int, a: int = _ALIGN) -> int:
    return (v + a - 1) // a * a


def sigma_schedule(sigma0: float, beta: float, sigma_min: float, it: int) -> float:
    return max(sigma0 * beta ** (0.5 * it), sigma_min)


def _workspace(nbytes: int, device) -> torch.Tensor:
    t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise RuntimeError("workspace is not 256-byte aligned")
    return t


class _Ticker:
    """Records (start, end) CUDA/HIP events around consecutive calls."""

    def __init__(self, marks):
        self.marks = marks
        self.name = None
        self.ev = None

    def _event(self):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def start(self, name):
        if self.marks is not None:
            self.name, self.ev = name, self._event()

    def next(self, name):
        if self.marks is not None:
            e = self._event()
            self.marks.setdefault(self.name, []).append((self.ev, e))
            self.name, self.ev = name, e

    def stop(self):
        if self.marks is not None:
            e = self._event()
            self.marks.setdefault(self.name, []).append((self.ev, e))


class GNMPPI:
    """Alg. 1 on the GPU.  ``sampler`` is "gaussian" (Method D, antithetic
    Philox normals) or "sigma_points" (Method E, the 2n-point Dirac mixture)."""

    def __init__(self, dprob: DeviceProblem, x0, settings, seed: int = 1, U0=None,
                 sampler: str = "gaussian", max_iters: int | None = None, overlap=False,
                 form_jacobian: bool = False, nominal_from_line: bool = False):
        self.p = dprob
        # form_jacobian: GetJacobian then the GGN step as two calls
        # (gnmppi_reconstruct_jacobian, gnmppi_ggn_step), J formed in HBM;
        # otherwise one gnmppi_ggn_direction call computes the same direction
        # from S = dR W^T without forming J = S G^{-1}, with G = W W^T from
        # the same contraction as S, on one stream (overlap is then unused).
        self.form_jacobian = bool(form_jacobian)
        # G = W W^T and its inverse depend only on W, and W only on the seed
        # and the iteration, so (LS estimator only) they can be factored on a
        # side stream that the main stream joins just before the first use
        # of G (J = S G^{-1}, or the direction's normal matrix).
        # overlap = "ahead" (or True): the side stream draws its own copy of
        # the next iteration's W and factors its G into a second workspace
        # while the main stream finishes the current iteration and rolls out
        # the next.  overlap = "prefetch": the same, and the main stream rolls
        # out with the side stream's W instead of drawing its own (it waits
        # for the side stream's sampler before the rollout; no sampler on the
        # main stream).  overlap =
        # "same": it forks after this iteration's sampler and factors G under
        # the rollout and S.  Which one is faster depends
        # on the sizes (the cross-stream edges of a graph cost a few us each);
        # inside a captured graph either beats a single stream, with eager
        # launches the waits cost more than the overlap saves, hence off by
        # default.
        if overlap not in (False, True, "ahead", "prefetch", "same"):
            raise ValueError("overlap must be False, True, 'ahead', 'prefetch' or 'same', "
                             f"not {overlap!r}")
        mode = "ahead" if overlap is True else overlap
        self.overlap = bool(mode) and settings.jacobian == "ls" and self.form_jacobian
        self.ahead = self.overlap and mode in ("ahead", "prefetch")
        self.prefetch = self.overlap and mode == "prefetch"
        self.side = torch.cuda.Stream(device=dprob.device) if self.overlap else None
        self.s = settings
        self.seed = int(seed)
        self.sampler = sampler
        n, m = dprob.n, dprob.m
        dev, dt = dprob.device, dprob.tdtype
        self.K = 2 * n if sampler == "sigma_points" else settings.K
        K = self.K
        self.n, self.m = n, m
        self.x0 = dprob.tensor(x0)
        self.U = torch.zeros(n, dtype=dt, device=dev) if U0 is None else dprob.tensor(U0)
        self.W = torch.zeros(n, _round_up(K), dtype=dt, device=dev)
        self.R = torch.zeros(m, _round_up(K), dtype=dt, device=dev)
        self.C = torch.zeros(K, dtype=dt, device=dev)
        self.r0 = torch.zeros(m, dtype=dt, device=dev)
        self.c0 = torch.zeros(1, dtype=dt, device=dev)
        self.J = torch.zeros(m, n, dtype=dt, device=dev) if self.form_jacobian else None
        self.dU = torch.zeros(n, dtype=dt, device=dev)
        self.alpha = torch.tensor([settings.gamma ** j for j in range(settings.n_alpha)],
                                  dtype=dt, device=dev)
        self.C_line = torch.zeros(settings.n_alpha, dtype=dt, device=dev)
        # nominal_from_line: the single-stream sampling path takes the nominal
        # residuals of the next iterate from the line search (its chosen
        # candidate is that iterate) instead of a nominal column in the next
        # rollout: one block less for the rollout, residual stores and a copy
        # more for the line search, which pays where the nominal column alone
        # would take a CU's second or third block (bench.py times both).
        # R_cand: scratch for the candidates' residual vectors
        self.nominal_from_line = (nominal_from_line and not self.form_jacobian
                                  and sampler == "gaussian")
        self.R_cand = (torch.zeros(settings.n_alpha * m, dtype=dt, device=dev)
                       if self.nominal_from_line else None)
        iters = max_iters if max_iters is not None else settings.iters
        self.info = torch.zeros(max(iters, 1), 3, dtype=torch.float64, device=dev)
        # status words per iteration: Jacobian (rank of G), GGN step (positive
        # definiteness; without J formed also the only check of G: a singular
        # G makes S^T S singular), G^{-1} factored on the side stream, line
        # search (a finite candidate); words that a path does not use stay 0
        self.status = torch.zeros(iters if iters else 1, 4, dtype=torch.int32, device=dev)
        code = _lib.F32 if dt == torch.float32 else _lib.F64
        # the direction call's workspace is the Jacobian workspace followed by
        # the GGN workspace
        wbytes = (_lib.gnmppi_jacobian_workspace(code, m, n, K) if self.form_jacobian
                  else _lib.gnmppi_ggn_direction_workspace(code, m, n, K))
        self.work_j = _workspace(wbytes, dev)
        self.works = [self.work_j]
        self.W_side = None
        if self.ahead:
            # iteration it uses works[it % 2]; the side stream fills the other
            self.works.append(_workspace(wbytes, dev))
            self.W_side = torch.zeros_like(self.W)
        self._gram_for = None  # iteration whose G^{-1} the side stream has been given
        self.work_g = (_workspace(_lib.gnmppi_ggn_workspace(code, m, n), dev) if self.form_jacobian
                       else None)
        self.method = _lib.JAC_LS if settings.jacobian == "ls" else _lib.JAC_MC
        if dt == torch.float32:
            self.method |= {"native": 0, "bf16x3": _lib.JAC_BF16X3,
                            "bf16": _lib.JAC_BF16}[settings.contraction]

    def sigma(self, it: int) -> float:
        s = self.s
        return sigma_schedule(s.sigma0, s.beta, s.sigma_min, it)

    def _sample(self, W, it: int):
        if self.sampler == "sigma_points":
            _lib.gnmppi_sigma_points(W, self.sigma(it))
        else:
            _lib.gnmppi_sample(W, self.sigma(it), self.seed, it, antithetic=self.s.antithetic,
                               K=self.K)

    def _side_gram(self, it: int, after=None):
        """Enqueues on the side stream: W of iteration ``it`` (the same draws
        as the main stream's, into W_side) and G^{-1} into works[it % 2].
        Ordered after the event ``after`` (J of iteration it - 1), else after
        all work enqueued so far on the current stream, so the last reads of
        that workspace (iteration it - 2) and of W_side (iteration it - 1,
        whose reads of W end with J) are done."""
        K = self.K
        if after is not None:
            self.side.wait_event(after)
        else:
            self.side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.side):
            W2 = self.W_side[:, :K]
            self._sample(W2, it)
            if self.prefetch:
                self._w_ready = torch.cuda.Event()
                self._w_ready.record()
            _lib.gnmppi_perturbation_gram(W2, self.works[it % 2], self.m, self.status[it, 2:3], K)
        self._gram_for = it

    def step(self, it: int, marks=None, ahead: bool = True, nominal: bool = True,
             keep_nominal: bool = False):
        """One iteration of Alg. 1: GetJacobian, full GGN step, line search,
        apply; the covariance shrink enters through ``sigma(it)``.  With
        ``marks`` (a dict name -> list), a pair of timing events is recorded
        around each library call on the current stream.  With overlap
        "ahead" and ``ahead``, the side stream's work for iteration it + 1 is
        enqueued once J of this iteration no longer needs the side stream.
        On the single-stream sampling path (``nominal_from_line``):
        ``keep_nominal`` has the line search write r0, c0 of the updated
        controls, and ``nominal=False`` rolls out without the nominal column,
        taking r0 from the previous step's line search -- for consecutive
        steps with no change of U in between."""
        K, sig = self.K, self.sigma(it)
        W = self.W[:, :K]
        work = self.works[it % 2] if self.ahead else self.work_j
        if self.ahead and self._gram_for != it:
            self._side_gram(it)  # not enqueued by a preceding step
        tick = _Ticker(marks)
        if not self.overlap and self.sampler == "gaussian":
            # one launch draws W and rolls out (residuals and the nominal
            # cost only: the step never reads C)
            tick.start("sample_rollout")
            skip = self.nominal_from_line and not nominal
            _lib.gnmppi_sample_rollout(self.p, self.x0, self.U, W, self.sigma(it), self.seed, it, K,
                                       antithetic=self.s.antithetic, R=self.R[:, :K],
                                       r0=None if skip else self.r0, c0=None if skip else self.c0)
        else:
            tick.start("sample")
            if self.prefetch:
                # W of this iteration comes from the side stream (its G^{-1} is
                # joined before J as in "ahead")
                torch.cuda.current_stream().wait_event(self._w_ready)
                W = self.W_side[:, :K]
            else:
                self._sample(W, it)
            if self.overlap and not self.ahead:
                sampled = torch.cuda.Event()
                sampled.record()
            tick.next("rollout")
            # residuals and the nominal cost only: the step never reads C
            _lib.gnmppi_rollout(self.p, self.x0, self.U, W, K, self.R[:, :K], None, self.r0,
                                self.c0)
            if self.overlap and not self.ahead:
                # enqueued after the rollout so that a captured graph keeps the
                # rollout on the sampling queue and forks only the W-only work
                self.side.wait_event(sampled)
                with torch.cuda.stream(self.side):
                    _lib.gnmppi_perturbation_gram(W, work, self.m, self.status[it, 2:3], K)
        tick.next("jacobian" if self.form_jacobian else "direction")
        j_done = None
        if not self.form_jacobian:
            self._direction(it, W, work, sig)
        elif self.overlap:
            # S = dR W^T needs only the rollout; the join with the side stream
            # comes just before J = S G^{-1}
            method = self.method | _lib.JAC_GRAM_READY
            _lib.gnmppi_reconstruct_jacobian(self.R[:, :K], self.r0, W, self.J, work,
                                             method | _lib.JAC_S_ONLY, sig * sig,
                                             self.status[it, 0:1], K)
            torch.cuda.current_stream().wait_stream(self.side)
            _lib.gnmppi_reconstruct_jacobian(self.R[:, :K], self.r0, W, self.J, work,
                                             method | _lib.JAC_APPLY_ONLY, sig * sig,
                                             self.status[it, 0:1], K)
            if self.ahead:
                if ahead and it + 1 < self.status.shape[0]:
                    # the next iteration's side work waits only for this J; it
                    # is enqueued after the rest of this iteration, so that a
                    # captured graph keeps the GGN step on J's queue
                    j_done = torch.cuda.Event()
                    j_done.record()
                else:
                    self._gram_for = None
        else:
            _lib.gnmppi_reconstruct_jacobian(self.R[:, :K], self.r0, W, self.J, self.work_j,
                                             self.method, sig * sig, self.status[it, 0:1], K)
        if self.form_jacobian:
            tick.next("ggn_step")
            _lib.gnmppi_ggn_step(self.J, self.r0, self.s.lm_lambda, self.dU, self.work_g,
                                 self.status[it, 1:2])
        tick.next("line_search")
        if self.nominal_from_line and keep_nominal:
            _lib.gnmppi_line_search_nominal(self.p, self.x0, self.U, self.dU, self.alpha,
                                            self.R_cand, self.r0, self.c0, self.C_line,
                                            self.info[it], self.status[it, 3:4])
        else:
            _lib.gnmppi_line_search(self.p, self.x0, self.U, self.dU, self.alpha, self.C_line,
                                    self.info[it], self.status[it, 3:4])
        tick.stop()
        if self.overlap and j_done is not None:
            self._side_gram(it + 1, after=j_done)

    def _direction(self, it: int, W, work, sig: float):
        """GetJacobian and the GGN step of iteration ``it`` as one
        gnmppi_ggn_direction call (J is not formed; for LS, G = W W^T comes
        out of the same contraction as S)."""
        _lib.gnmppi_ggn_direction(self.R[:, :self.K], self.r0, W, self.dU, work, self.method,
                                  sig * sig, self.s.lm_lambda, self.status[it, 1:2], K=self.K)

    def capture(self, iters: int, it0: int = 0):
        """Captures iterations it0 .. it0 + iters - 1 into one HIP graph.

        Every call only enqueues kernels on the current stream and the
        iteration-dependent arguments (sampling scale, Philox stream, output
        rows) are fixed at capture, so ``graph.replay()`` re-runs exactly these
        iterations from the current U with a single launch.  The graph owns no
        memory of its own: all buffers belong to this solver."""
        side = torch.cuda.Stream(device=self.p.device)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up outside capture, as torch requires
            self.step(it0, ahead=False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            # the first iteration enqueues its own side-stream work; the last
            # enqueues none, so every fork is joined inside the graph.  Only
            # the first rolls out the nominal column (U may have changed
            # between replays); each later one takes r0 from the line search
            # before it
            for it in range(it0, it0 + iters):
                self.step(it, ahead=it + 1 < it0 + iters, nominal=it == it0,
                          keep_nominal=it + 1 < it0 + iters)
        self._gram_for = None
        return graph

    def solve(self, iters: int | None = None, events: bool = False):
        """Runs ``iters`` iterations; returns (costs, alphas, statuses, event list)."""
        iters = self.s.iters if iters is None else iters
        evs = []
        if events:
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record()
            evs.append(e0)
        for it in range(iters):
            self.step(it, ahead=it + 1 < iters, nominal=it == 0, keep_nominal=it + 1 < iters)
            if events:
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                evs.append(e)
        return evs

    def history(self, iters: int):
        info = self.info[:iters].cpu()
        return info[:, 1].double().numpy(), info[:, 0].double().numpy(), self.status[:iters].cpu().numpy()


# Iteration schedules of GNMPPI: "direct" -- one gnmppi_ggn_direction call per
# iteration (J not formed), one stream; "direct-line" -- the same, and in a
# run of steps the line search hands the next step its nominal residuals
# (gnmppi_line_search_nominal) so that rollout leaves out the nominal column;
# "formed" -- J formed (gnmppi_reconstruct_jacobian, then gnmppi_ggn_step),
# one stream; "ahead", "prefetch", "same" -- J formed, with G^{-1} factored on
# a side stream.  Values: (form J, side-stream mode, nominal from the line
# search).
SCHEDULES = {"direct": (False, False, False), "direct-line": (False, False, True),
             "formed": (True, False, False), "ahead": (True, "ahead", False),
             "prefetch": (True, "prefetch", False), "same": (True, "same", False)}


def make_solver(dprob: DeviceProblem, x0, settings, schedule: str = "direct", **kw) -> GNMPPI:
    """GNMPPI with the iteration schedule ``schedule`` (a key of SCHEDULES)."""
    form, overlap, line_nominal = SCHEDULES[schedule]
    return GNMPPI(dprob, x0, settings, overlap=overlap, form_jacobian=form,
                  nominal_from_line=line_nominal, **kw)


class PlainMPPI:
    """Method C: U <- U + sum_s w_s W_s / sum_s w_s (Eqs. (7)-(8)).  The
    rollout of each iteration also evaluates the nominal U, so cost[it] holds
    C(U_it) without an extra launch."""

    def __init__(self, dprob: DeviceProblem, x0, settings, seed: int = 2, U0=None,
                 max_iters: int = 1000):
        self.p = dprob
        self.s = settings
        self.seed = int(seed)
        n = dprob.n
        dev, dt = dprob.device, dprob.tdtype
        K = settings.K
        self.K = K
        self.x0 = dprob.tensor(x0)
        self.U = torch.zeros(n, dtype=dt, device=dev) if U0 is None else dprob.tensor(U0)
        self.W = torch.zeros(n, _round_up(K), dtype=dt, device=dev)
        self.C = torch.zeros(K, dtype=dt, device=dev)
        self.cost = torch.zeros(max_iters + 1, dtype=dt, device=dev)
        self.status = torch.zeros(max_iters + 1, dtype=torch.int32, device=dev)
        self.sigma0 = settings.mppi_sigma0 or settings.sigma0

    def sigma(self, it: int) -> float:
        return sigma_schedule(self.sigma0, self.s.mppi_beta, 0.0, it)

    def step(self, it: int):
        K = self.K
        W = self.W[:, :K]
        _lib.gnmppi_sample(W, self.sigma(it), self.seed, it, antithetic=self.s.antithetic, K=K)
        _lib.gnmppi_rollout(self.p, self.x0, self.U, W, K, None, self.C, None, self.cost[it:it + 1])
        _lib.gnmppi_mppi_update(self.C, W, self.s.temperature, self.U, None,
                                self.status[it:it + 1], K)

    def final_cost(self, it: int):
        """Enqueues the nominal rollout of the current U into cost[it]."""
        _lib.gnmppi_rollout(self.p, self.x0, self.U, None, 0, None, None, None,
                            self.cost[it:it + 1])
