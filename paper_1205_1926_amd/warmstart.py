"""Learned warm start of the dual PCGP: the perceptron on the device, data
collection from converged load steps, training and evaluation.

Every arithmetic step (features, forward, loss, gradients, Adam, candidate)
runs in the HIP library; this module holds device buffers and the loop.

The network maps features of an interface node (load-increment direction,
the node's multipliers of the last converged load step, the hardening of the
elements around it, its class) to the change of the node's multipliers over
the next load step, both scaled by the nodal force of the increment.  The
library offers the resulting candidate beside the previous Newton
iteration's multipliers and keeps whichever has the smaller projected
initial residual, so a poor prediction costs one F-apply and nothing else.

Command line (data generation on seeded loads, training, evaluation on
unseen seeds)::

    python -m paper_1205_1926_amd.warmstart --config 3 --train-seeds 0:100 \\
        --test-seeds 1000:1003 --epochs 4 --out weights.safetensors --report r.json
"""

from __future__ import annotations

import argparse
import ctypes as C
import json
import sys
import time

import numpy as np

from . import _capi as A

D_IN, D_H, D_OUT = 31, 256, 21


def _torch():
    import torch
    return torch


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class WarmNet:
    """Device copy of the perceptron: FP32 master weights, bf16 shadows,
    gradients and Adam moments.  ``params``: dict of numpy arrays W1..W3
    (out x in) and b1..b3."""

    def __init__(self, params, device: str = "cuda:0", stream=None):
        torch = _torch()
        self.lib = A.load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.dims = (params["W1"].shape[1], params["W1"].shape[0], params["W2"].shape[0], params["W3"].shape[0])
        if self.dims[1] != self.dims[2]:
            raise ValueError("hidden layers must have equal width")
        f32 = dict(dtype=torch.float32, device=self.device)
        self.W = [torch.tensor(np.asarray(params[f"W{l + 1}"], dtype=np.float32), **f32).contiguous()
                  for l in range(3)]
        self.b = [torch.tensor(np.asarray(params[f"b{l + 1}"], dtype=np.float32), **f32).contiguous()
                  for l in range(3)]
        self.Wb = [torch.empty(w.shape, dtype=torch.int16, device=self.device) for w in self.W]
        z = lambda ts: [torch.zeros_like(t) for t in ts]
        self.gW, self.gb = z(self.W), z(self.b)
        self.mW, self.vW, self.mb, self.vb = z(self.W), z(self.W), z(self.b), z(self.b)
        s = A.Mlp()
        s.d_in, s.d_h, s.d_out = self.dims[0], self.dims[1], self.dims[3]
        for name in ("W", "b", "Wb", "gW", "gb", "mW", "vW", "mb", "vb"):
            arr = getattr(s, name)
            for l, t in enumerate(getattr(self, name)):
                arr[l] = t.data_ptr()
        self.s = s
        self.step = 0
        self._work = None
        self._loss = torch.zeros(1, **f32)
        self._check(self.lib.tfeti_mlp_sync_bf16(C.byref(s), self._st()), "mlp_sync_bf16")

    def _st(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _check(self, rc, what):
        if rc < 0:
            raise A.TfetiError(f"{what}: {rc}")

    def _work_for(self, n):
        torch = _torch()
        fl = C.c_int64()
        self._check(self.lib.tfeti_mlp_work_size(C.byref(self.s), n, C.byref(fl)), "mlp_work_size")
        if self._work is None or self._work.numel() < fl.value:
            self._work = torch.empty(int(fl.value), dtype=torch.float32, device=self.device)
        return self._work

    def forward(self, X, Y=None):
        torch = _torch()
        n = X.shape[0]
        if Y is None:
            Y = torch.empty((n, self.dims[3]), dtype=torch.float32, device=self.device)
        work = self._work_for(n)
        self._check(self.lib.tfeti_mlp_forward(C.byref(self.s), n, _p(X), _p(Y), _p(work), self._st()),
                    "mlp_forward")
        return Y

    def loss_grad(self, X, T, M, Y=None):
        """Forward, masked MSE and gradients; returns (loss device scalar, Y)."""
        torch = _torch()
        n = X.shape[0]
        if Y is None:
            Y = torch.empty((n, self.dims[3]), dtype=torch.float32, device=self.device)
        work = self._work_for(n)
        self._check(self.lib.tfeti_mlp_loss_grad(C.byref(self.s), n, _p(X), _p(T), _p(M), _p(Y), _p(self._loss),
                                                 _p(work), self._st()), "mlp_loss_grad")
        return self._loss, Y

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        self._check(self.lib.tfeti_mlp_adam(C.byref(self.s), self.step, C.c_float(lr), C.c_float(beta1),
                                            C.c_float(beta2), C.c_float(eps), self._st()), "mlp_adam")

    # ------------------------------------------------------------------ host copies
    def params(self):
        out = {}
        for l in range(3):
            out[f"W{l + 1}"] = self.W[l].double().cpu().numpy()
            out[f"b{l + 1}"] = self.b[l].double().cpu().numpy()
        return out

    def grads(self):
        out = {}
        for l in range(3):
            out[f"W{l + 1}"] = self.gW[l].double().cpu().numpy()
            out[f"b{l + 1}"] = self.gb[l].double().cpu().numpy()
        return out

    def bf16_weights(self):
        """The bf16 shadow weights the products use, widened to float64."""
        out = {}
        for l in range(3):
            u = self.Wb[l].cpu().numpy().view(np.uint16).astype(np.uint32) << 16
            out[f"W{l + 1}"] = u.view(np.float32).astype(np.float64)
        return out

    def save(self, path):
        from safetensors.torch import save_file
        t = {}
        for l in range(3):
            t[f"W{l + 1}"] = self.W[l].cpu()
            t[f"b{l + 1}"] = self.b[l].cpu()
        save_file(t, path)

    @classmethod
    def load(cls, path, device="cuda:0", stream=None):
        from safetensors.numpy import load_file
        return cls(load_file(path), device=device, stream=stream)


class PreviousStep:
    """Stand-in network that predicts no change: the candidate is the last
    converged step's multipliers themselves (the baseline a trained network
    has to beat)."""

    def forward(self, X):
        torch = _torch()
        return torch.zeros((X.shape[0], D_OUT), dtype=torch.float32, device=X.device)


# ---------------------------------------------------------------------- solver glue
def propose(solver, net, dload):
    """Learned candidate for the load step about to run: lambda_conv + s * net(features).
    Sets it on the solver and returns it (None before the first committed step)."""
    lam_c, ok = solver.converged_lambda()
    if not ok:
        solver.set_learned_guess(None)
        return None
    X, _ = solver.warm_features(lam_c, dload, want_mask=False)
    Y = net.forward(X)
    cand = solver.warm_candidate(lam_c, Y, dload)
    solver.set_learned_guess(cand)
    return cand


def run_step(solver, net=None, record=False):
    """One load step (Newton to convergence, commit).  With ``net`` the
    learned candidate is offered; with ``record`` the features before the
    step and the targets after it are returned as (X, T), or None on the
    first step.  Returns (newton reports, sample)."""
    dload = solver.load_increment()
    lam_c, ok = solver.converged_lambda()
    X = None
    if record and ok:
        X, _ = solver.warm_features(lam_c, dload, want_mask=False)
    if net is not None:
        propose(solver, net, dload)
    hist = solver.load_step()
    sample = None
    if record and ok:
        lam_n, _ = solver.converged_lambda()
        sample = (X, solver.warm_targets(lam_c, lam_n, dload))
    return hist, sample


def mask(solver):
    """Slot mask (n x 21) of the solver's interface nodes."""
    _, M = solver.warm_features(None, 1.0)
    return M


def train(net, samples, M, epochs=1, batch=4096, lr=1e-3, seed=0, log_every=200, log=None):
    """Adam on mini-batches of contiguous node ranges drawn in a seeded random
    order from every sample (X, T); M is the shared slot mask.  Returns the
    mean loss of each epoch."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    n = M.shape[0]
    starts = list(range(0, n, batch))
    losses = []
    for ep in range(epochs):
        acc = torch.zeros(1, dtype=torch.float64, device=net.device)
        count = 0
        order = [(i, s) for i in range(len(samples)) for s in starts]
        for j in rng.permutation(len(order)):
            i, s = order[j]
            X, T = samples[i]
            e = min(n, s + batch)
            loss, _ = net.loss_grad(X[s:e], T[s:e], M[s:e])
            net.adam(lr=lr)
            acc += loss.double()
            count += 1
            if log and count % log_every == 0:
                log(f"epoch {ep} batch {count}/{len(order)} loss {float(loss):.4e}")
        losses.append(float(acc) / max(count, 1))
        if log:
            log(f"epoch {ep} mean loss {losses[-1]:.4e}")
    return losses


def eval_loss(net, samples, M, batch=65536):
    torch = _torch()
    tot = torch.zeros(1, dtype=torch.float64, device=net.device)
    cnt = 0
    n = M.shape[0]
    for X, T in samples:
        for s in range(0, n, batch):
            e = min(n, s + batch)
            loss, _ = net.loss_grad(X[s:e], T[s:e], M[s:e])
            tot += loss.double() * (e - s)
            cnt += e - s
    return float(tot) / max(cnt, 1)


def path_stats(hists):
    """PCG iterations, F-applies and Newton-step time per Newton iteration index."""
    by_i = {}
    for hist in hists:
        for r in hist:
            d = by_i.setdefault(r["iteration"], dict(n=0, pcg_iters=0, fapplies=0, ms=0.0, learned=0))
            d["n"] += 1
            d["pcg_iters"] += r["pcg_iters"]
            d["fapplies"] += r["fapplies"]
            d["ms"] += r["ms_total"]
            d["learned"] += 1 if r.get("warm_choice") == 2 else 0
    tot = dict(pcg_iters=sum(d["pcg_iters"] for d in by_i.values()),
               fapplies=sum(d["fapplies"] for d in by_i.values()),
               newton_iters=sum(d["n"] for d in by_i.values()),
               ms=sum(d["ms"] for d in by_i.values()))
    return dict(total=tot, by_iteration={str(k): v for k, v in sorted(by_i.items())})


# ---------------------------------------------------------------------- command line
def _seeds(spec):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


def main(argv=None):
    import torch
    import workloads as W

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--train-seeds", default="0:100")
    ap.add_argument("--test-seeds", default="1000:1003")
    ap.add_argument("--steps", type=int, default=0, help="load steps per run (0: the workload's)")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--weights", default=None, help="skip training, evaluate these weights")
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    from .solver import GpuSolver
    dev = "cuda:0"
    rep = dict(config=a.config, train_seeds=a.train_seeds, test_seeds=a.test_seeds)
    mk = lambda seed: W.config(a.config, load_seed=seed)
    opts = dict(use_graph=1)
    if a.precision:
        opts["precision"] = a.precision
    if a.weights:
        net = WarmNet.load(a.weights, device=dev)
    else:
        net = WarmNet(W.mlp_init(a.init_seed), device=dev)
        samples, M = [], None
        t0 = time.time()
        for seed in _seeds(a.train_seeds):
            w = mk(seed)
            g = GpuSolver(w, device=dev, **opts)
            if M is None:
                M = mask(g)
            for _ in range(a.steps or w.steps):
                _, smp = run_step(g, record=True)
                if smp is not None:
                    samples.append(smp)
            g.close()
            log(f"seed {seed}: {len(samples)} samples, {time.time() - t0:.0f} s")
        rep["samples"] = len(samples)
        rep["nodes"] = int(M.shape[0])
        rep["data_s"] = time.time() - t0
        t1 = time.time()
        rep["init_loss"] = eval_loss(net, samples, M)
        rep["epoch_loss"] = train(net, samples, M, epochs=a.epochs, batch=a.batch, lr=a.lr,
                                  seed=a.init_seed, log=log)
        torch.cuda.synchronize()
        rep["train_s"] = time.time() - t1
        if a.out:
            net.save(a.out)
        del samples
    # evaluation on unseen loads: the same runs with and without the candidate
    ev = []
    for seed in _seeds(a.test_seeds):
        w = mk(seed)
        res = {}
        for name, use in (("fallback", None), ("previous_step", PreviousStep()), ("learned", net)):
            g = GpuSolver(w, device=dev, **opts)
            hists = []
            test_samples = []
            for _ in range(a.steps or w.steps):
                h, smp = run_step(g, net=use, record=(use is None))
                hists.append(h)
                if smp is not None:
                    test_samples.append(smp)
            res[name] = path_stats(hists)
            if use is None and test_samples:
                res["test_loss"] = eval_loss(net, test_samples, mask(g))
                res["zero_loss"] = float(sum(float((0.5 * (T * T).sum() / T.shape[0])) for _, T in test_samples)
                                         / len(test_samples))
            g.close()
        log(f"test seed {seed}: " + " ".join(f"{k} {res[k]['total']}" for k in ("fallback", "previous_step", "learned")))
        ev.append(dict(seed=seed, **res))
    rep["eval"] = ev
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
    log(json.dumps({k: v for k, v in rep.items() if k != "eval"}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
