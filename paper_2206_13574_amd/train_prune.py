"""Training of the diagonal keep/drop network used by the learned pruning
mode, and calibration of its keep threshold.

Data.  Exact runs (Algorithms 1-3) of the library with its trace dump on
synthetic bubble graphs shaped like the 5 kb test graph (SNP bubbles every
~100 bp, indel bubbles every ~500 bp with 1-20 bp arms), graph seeds 501,
502, ...; per graph 1 kb reads at a per-read error rate drawn from U(1%, 10%).
Every wavefront entry of every expanded score is one sample: its eight
features, and the label "lies on an optimal alignment" from the library's
host reverse recurrence (gwfa_label_entries).  Collection stops at the
requested number of samples.

Training.  Weighted binary cross-entropy (positives weighted by the
negative/positive ratio, capped), Adam on float32 master weights with the
bfloat16 copy used by every forward pass, all in the library's HIP kernels.
The feature scales map each feature's 99.9th percentile of |f| to 1.

Calibration.  On held-out graphs (seeds 601, 602, ...) of the same shape the
keep threshold is the largest one (most pruning) whose runs leave at most
`target` of the reads above their exact distance; exact and learned runs
are both made by the library.

Output: an .npz with the bfloat16 weights (uint16 bit patterns), the feature
scales, the threshold, the gate and period to use, and a JSON summary.
Usage: python -m paper_2206_13574_amd.train_prune --out path.npz
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import gwfa, synth

N_PARAM = gwfa.MLP_N
O_W1, O_B1, O_W2, O_B2, O_W3, O_B3 = 0, 512, 576, 4672, 4736, 4800
DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "prune_mlp.npz")


def log(msg):
    print(f"[train] {msg}", flush=True)


def train_graph(seed: int):
    return synth.bubble_graph(seed, 5000, snp_gap=100, indel_gap=500, indel_arm=(1, 20))


def train_reads(g, seed: int, n: int, read_len: int = 1000):
    return synth.sample_reads(g, seed, n, read_len, lambda rng, k: rng.uniform(0.01, 0.10, k))


def collect(ctx, seeds, reads_per_graph: int, target: int, read_len: int = 1000):
    """Samples from exact runs: features [N, 8] float32, labels [N] uint8."""
    feats, labels = [], []
    total, pos = 0, 0
    for gs in seeds:
        g = train_graph(gs)
        r = train_reads(g, gs + 100000, reads_per_graph, read_len)
        graph = gwfa.Graph.of(ctx, g)
        res, d, produced = gwfa.align_dump(ctx, graph, r.seq, r.off, r.v_start, gwfa.opts(traceback=False),
                                           dump_cap=1 << 23)
        graph.close()
        if produced > (1 << 23):
            raise RuntimeError("trace dump overflow; lower reads_per_graph")
        ok = res["status"] == gwfa.ST_OK
        keep = ok[d["read"]]
        d = {k: v[keep] for k, v in d.items()}
        cost, lab, dist = gwfa.label_entries(g, r.seq, r.off, r.v_start, d["read"], d["score"], d["i"], d["v"],
                                             d["off"])
        if not np.array_equal(dist[ok], res["dist"][ok]):
            raise RuntimeError("label recurrence and alignment disagree on d*")
        feats.append(d["feat"])
        labels.append(lab)
        total += len(lab)
        pos += int(lab.sum())
        log(f"graph {gs}: {len(lab)} samples ({lab.mean():.4f} positive); total {total}")
        if total >= target:
            break
    f = np.concatenate(feats)[:target]
    y = np.concatenate(labels)[:target]
    return f, y


def init_params(rng) -> np.ndarray:
    w = np.zeros(N_PARAM, dtype=np.float32)
    w[O_W1:O_B1] = rng.normal(0.0, np.sqrt(2.0 / 8), 512)
    w[O_W2:O_B2] = rng.normal(0.0, np.sqrt(2.0 / 64), 4096)
    w[O_W3:O_B3] = rng.normal(0.0, np.sqrt(1.0 / 64), 64)
    return w


def to_bf16_bits(w: np.ndarray) -> np.ndarray:
    """float -> bfloat16 bit patterns (nearest, ties to even)."""
    u = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def feature_scale(f: np.ndarray) -> np.ndarray:
    q = np.quantile(np.abs(f), 0.999, axis=0)
    return (1.0 / np.maximum(q, 1e-3)).astype(np.float32)


class Trainer:
    def __init__(self, ctx, scale: np.ndarray, w0: np.ndarray):
        torch = ctx.torch
        self.ctx, self.torch, self.scale = ctx, torch, scale
        dev = ctx.tdev
        self.master = torch.from_numpy(w0.astype(np.float32)).to(dev)
        self.m1 = torch.zeros(N_PARAM, dtype=torch.float32, device=dev)
        self.m2 = torch.zeros(N_PARAM, dtype=torch.float32, device=dev)
        self.wb = torch.zeros(N_PARAM, dtype=torch.int16, device=dev)
        self.grad = torch.zeros(N_PARAM, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        gwfa.mlp_cast_dev(ctx, self.master, self.wb)
        self.step = 0

    def fit(self, f: np.ndarray, y: np.ndarray, epochs: int, batch: int, lr: float, pos_weight: float, seed: int):
        torch, ctx = self.torch, self.ctx
        rng = np.random.default_rng(seed)
        perm = rng.permutation(len(y))
        tf = torch.from_numpy(np.ascontiguousarray(f[perm])).to(ctx.tdev)
        ty = torch.from_numpy(np.ascontiguousarray(y[perm])).to(ctx.tdev)
        nb = (len(y) + batch - 1) // batch
        for ep in range(epochs):
            t0 = time.time()
            lsum = 0.0
            lr_ep = lr * (0.5 ** max(0, ep - epochs // 2))
            for bi in rng.permutation(nb):
                a = int(bi) * batch
                b = min(len(y), a + batch)
                gwfa.mlp_grad_dev(ctx, tf[a:b], ty[a:b], self.scale, self.wb, self.grad, self.loss,
                                  pos_weight=pos_weight)
                self.step += 1
                gwfa.mlp_adam_dev(ctx, self.master, self.m1, self.m2, self.grad, self.wb, self.step, lr_ep)
                lsum += float(self.loss.item()) * (b - a)
            log(f"epoch {ep}: loss {lsum / len(y):.5f} lr {lr_ep:.2e} ({time.time() - t0:.1f} s)")

    def weights_bf16(self) -> np.ndarray:
        return self.wb.cpu().numpy().view(np.uint16).copy()

    def logits(self, f: np.ndarray) -> np.ndarray:
        torch, ctx = self.torch, self.ctx
        tf = torch.from_numpy(np.ascontiguousarray(f)).to(ctx.tdev)
        out = torch.zeros(len(f), dtype=torch.float32, device=ctx.tdev)
        gwfa.mlp_logits_dev(ctx, tf, self.scale, self.wb, out)
        return out.cpu().numpy()


def exact_and_learned(ctx, graphs_reads, w_bf16, scale, taus, gate: int, period: int):
    """Fraction of reads above the exact distance and total work per tau."""
    ctx.mlp_load(w_bf16, scale)
    over = np.zeros(len(taus))
    work = np.zeros(len(taus))
    n_reads, work_exact = 0, 0
    for g, r in graphs_reads:
        graph = gwfa.Graph.of(ctx, g)
        ex, _ = gwfa.align(ctx, graph, r.seq, r.off, r.v_start, gwfa.opts(traceback=False))
        n_reads += r.n
        work_exact += int(ex["work"].sum())
        for t, tau in enumerate(taus):
            lr_, _ = gwfa.align(ctx, graph, r.seq, r.off, r.v_start,
                                gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=float(tau), mlp_gate=gate,
                                          mlp_period=period, traceback=False))
            if (lr_["dist"] < ex["dist"]).any():
                raise RuntimeError("a pruned run went below the exact distance")
            over[t] += int((lr_["dist"] > ex["dist"]).sum())
            work[t] += int(lr_["work"].sum())
        graph.close()
    return over / n_reads, work / max(work_exact, 1)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--samples", type=int, default=10_000_000)
    ap.add_argument("--reads-per-graph", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=32768)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--pos-weight-cap", type=float, default=20.0)
    ap.add_argument("--calib-graphs", type=int, default=6)
    ap.add_argument("--calib-reads", type=int, default=200)
    ap.add_argument("--target", type=float, default=0.005, help="largest fraction of calibration reads over exact")
    ap.add_argument("--gate", type=int, default=32)
    ap.add_argument("--period", type=int, default=4)
    ap.add_argument("--seed", type=int, default=12345)
    a = ap.parse_args(argv)
    t_start = time.time()
    ctx = gwfa.Context(0)
    f, y = collect(ctx, range(501, 601), a.reads_per_graph, a.samples)
    n_pos = int(y.sum())
    pos_weight = float(min(a.pos_weight_cap, (len(y) - n_pos) / max(n_pos, 1)))
    scale = feature_scale(f)
    log(f"{len(y)} samples, {n_pos} positive, pos_weight {pos_weight:.2f}, scale {np.round(scale, 4).tolist()}")
    rng = np.random.default_rng(a.seed)
    tr = Trainer(ctx, scale, init_params(rng))
    tr.fit(f, y, a.epochs, a.batch, a.lr, pos_weight, a.seed + 1)
    w = tr.weights_bf16()
    # held-out calibration
    calib = []
    for k in range(a.calib_graphs):
        g = train_graph(601 + k)
        calib.append((g, train_reads(g, 701 + k, a.calib_reads)))
    z = tr.logits(f[:: max(1, len(f) // 200000)])
    taus = np.unique(np.round(np.quantile(z, np.linspace(0.05, 0.95, 19)), 3))
    over, work = exact_and_learned(ctx, calib, w, scale, taus, a.gate, a.period)
    for t, o, wk in zip(taus, over, work):
        log(f"tau {t:+.3f}: reads over exact {o:.4f}, work vs exact {wk:.3f}")
    ok = over <= a.target
    tau = float(taus[ok].max()) if ok.any() else float(taus.min())
    log(f"chosen tau {tau:+.3f}")
    meta = dict(samples=int(len(y)), positives=n_pos, pos_weight=pos_weight, epochs=a.epochs, batch=a.batch,
                lr=a.lr, train_graph_seeds="501..", calib_graph_seeds=f"601..{600 + a.calib_graphs}",
                calib_reads=a.calib_graphs * a.calib_reads, target=a.target,
                calib=[dict(tau=float(t), over=float(o), work=float(wk)) for t, o, wk in zip(taus, over, work)],
                seconds=round(time.time() - t_start, 1))
    np.savez(a.out, w_bf16=w, scale=scale, tau=np.float32(tau), gate=np.int32(a.gate), period=np.int32(a.period),
             meta=np.array(json.dumps(meta)))
    log(f"wrote {a.out}")
    ctx.close()


def load(path: str = DEFAULT_PATH) -> dict:
    """Trained weights and settings (no pickled objects)."""
    z = np.load(path, allow_pickle=False)
    return dict(w_bf16=z["w_bf16"].astype(np.uint16), scale=z["scale"].astype(np.float32), tau=float(z["tau"]),
                gate=int(z["gate"]), period=int(z["period"]), meta=json.loads(str(z["meta"])))


if __name__ == "__main__":
    main()
