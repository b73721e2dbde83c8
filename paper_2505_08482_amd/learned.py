"""Learned fine-level start of the sound speed (replacing the linear
interpolation of the coarse iterate that starts a finer multigrid level,
Sec. 3.1), trained on the GPU by the library's own layer kernels.

The network (a U-Net with 4 resolutions, ``base`` = 32 channels at the top,
3x3 convolutions, ReLU, 2x2 average pooling, nearest upsampling, skip
connections, a 1x1 head) reads the interpolated coarse sound speed and the
interpolated sum over datasets of the initial-pressure gradient, and proposes
a correction added to the interpolated sound speed; the result is projected
onto the bounds of eq. (11).  Plain gradient iterations continue from it, so
the reconstruction still decides the final c and remains the fallback.

Every layer runs in ``libpat.so`` (``include/pat_nn.h``); this module owns the
parameter layout, the buffers and the order of the layer calls.  Weights are
bfloat16 for the kernels with float32 master copies for Adam.
"""
from __future__ import annotations

import dataclasses
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import inputs as I
from . import nn, pat

LEVELS = 4
CIN = 8            # input channels: (c, gradient sum, 6 zero channels)
C_SHIFT = 1500.0   # m/s: input channel 0 is (c - C_SHIFT) / C_SCALE
C_SCALE = 100.0    # m/s: the output is a correction in units of C_SCALE


def layer_table(cin: int, base: int) -> List[Tuple[str, int, int]]:
    """``(name, C_in, C_out)`` of the 3x3 convolutions in forward order:
    encoder ``e{l}a, e{l}b`` (l = 0..3), decoder ``d{l}a, d{l}b`` (l = 2, 1, 0);
    decoder inputs are ``[skip, upsampled]`` concatenations."""
    ch = [base << l for l in range(LEVELS)]
    table = []
    c = cin
    for l in range(LEVELS):
        table.append((f"e{l}a", c, ch[l]))
        table.append((f"e{l}b", ch[l], ch[l]))
        c = ch[l]
    for l in range(LEVELS - 2, -1, -1):
        table.append((f"d{l}a", ch[l] + ch[l + 1], ch[l]))
        table.append((f"d{l}b", ch[l], ch[l]))
    return table


class UNet:
    """Parameters in one flat float32 buffer (per layer: weights [cout][9][cin],
    then biases; the head's weights [base] and bias last), its bfloat16 copy,
    gradients and Adam moments of the same layout."""

    def __init__(self, base: int = 32, cin: int = CIN, seed: int = 0, device: str = "cuda"):
        if cin % 8 or base % 8:
            raise ValueError("channel counts must be multiples of 8")
        self.base, self.cin, self.device = base, cin, device
        self.table = layer_table(cin, base)
        self.shapes = {name: (ci, co) for name, ci, co in self.table}
        self.offsets: Dict[str, Tuple[int, int, int]] = {}
        off = 0
        for name, ci, co in self.table:
            self.offsets[name] = (off, off + co * 9 * ci, co)
            off += co * 9 * ci + co
        self.head_off = off
        self.n = off + base + 1
        rng = np.random.default_rng(seed)
        w = np.zeros(self.n, dtype=np.float32)
        for name, ci, co in self.table:
            o, ob, _ = self.offsets[name]
            w[o:ob] = rng.standard_normal(co * 9 * ci) * np.sqrt(2.0 / (9 * ci))   # He-normal
        self.w32 = torch.from_numpy(w).to(device)
        self.wbf = torch.empty(self.n, dtype=torch.bfloat16, device=device)
        self.grad = torch.zeros(self.n, dtype=torch.float32, device=device)
        self.m = torch.zeros_like(self.grad)
        self.v = torch.zeros_like(self.grad)
        self.step = 0
        self.sync_bf16()
        self._bufs: Dict[Tuple[int, int, int], Dict] = {}
        self._flip: Dict[str, torch.Tensor] = {}

    # -- parameter views ----------------------------------------------------
    def sync_bf16(self) -> None:
        nn.to_bf16(self.w32, self.wbf)

    def weight(self, name: str) -> torch.Tensor:
        o, ob, co = self.offsets[name]
        ci = self.shapes[name][0]
        return self.wbf[o:ob].view(co, 9, ci)

    def bias(self, name: str) -> torch.Tensor:
        _, ob, co = self.offsets[name]
        return self.w32[ob:ob + co]

    def grad_views(self, name: str):
        o, ob, co = self.offsets[name]
        return self.grad[o:ob], self.grad[ob:ob + co]

    def head_w(self) -> torch.Tensor:
        return self.wbf[self.head_off:self.head_off + self.base]

    def head_b(self) -> torch.Tensor:
        return self.w32[self.head_off + self.base:self.head_off + self.base + 1]

    def state(self) -> Dict[str, np.ndarray]:
        """Float32 master parameters by name (``<layer>.w``, ``<layer>.b``, ``head.w``, ``head.b``)."""
        w = self.w32.cpu().numpy()
        out = {}
        for name, ci, co in self.table:
            o, ob, _ = self.offsets[name]
            out[name + ".w"] = w[o:ob].reshape(co, 9, ci).copy()
            out[name + ".b"] = w[ob:ob + co].copy()
        out["head.w"] = w[self.head_off:self.head_off + self.base].copy()
        out["head.b"] = w[self.head_off + self.base:].copy()
        return out

    def load(self, state: Dict[str, np.ndarray]) -> None:
        w = np.zeros(self.n, dtype=np.float32)
        for name, ci, co in self.table:
            o, ob, _ = self.offsets[name]
            w[o:ob] = np.asarray(state[name + ".w"], dtype=np.float32).reshape(-1)
            w[ob:ob + co] = np.asarray(state[name + ".b"], dtype=np.float32).reshape(-1)
        w[self.head_off:self.head_off + self.base] = np.asarray(state["head.w"], dtype=np.float32).reshape(-1)
        w[self.head_off + self.base:] = np.asarray(state["head.b"], dtype=np.float32).reshape(-1)
        self.w32.copy_(torch.from_numpy(w))
        self.sync_bf16()

    # -- buffers --------------------------------------------------------------
    def buffers(self, B: int, H: int, W: int) -> Dict:
        key = (B, H, W)
        if key in self._bufs:
            return self._bufs[key]
        if H % (1 << (LEVELS - 1)) or W % (1 << (LEVELS - 1)):
            raise ValueError(f"H and W must be multiples of {1 << (LEVELS - 1)}")
        dev, bf = self.device, torch.bfloat16
        ch = [self.base << l for l in range(LEVELS)]
        res = [(H >> l, W >> l) for l in range(LEVELS)]

        def act(l, c):
            return torch.empty((B, res[l][0], res[l][1], c), dtype=bf, device=dev)

        b: Dict = {"act": {}, "grad": {}}
        A, G = b["act"], b["grad"]
        for l in range(LEVELS):
            if l > 0:
                A[f"in{l}"] = act(l, ch[l - 1])
                G[f"in{l}"] = act(l, ch[l - 1])
            A[f"e{l}a"] = act(l, ch[l])
            G[f"e{l}a"] = act(l, ch[l])
        for l in range(LEVELS - 1):
            A[f"cat{l}"] = act(l, ch[l] + ch[l + 1])
            G[f"cat{l}"] = act(l, ch[l] + ch[l + 1])
            A[f"e{l}b"] = A[f"cat{l}"][..., :ch[l]]          # skip half of the concatenation
            G[f"e{l}b"] = G[f"cat{l}"][..., :ch[l]]
            A[f"d{l}a"] = act(l, ch[l])
            G[f"d{l}a"] = act(l, ch[l])
            A[f"d{l}b"] = act(l, ch[l])
            G[f"d{l}b"] = act(l, ch[l])
        A[f"e{LEVELS - 1}b"] = act(LEVELS - 1, ch[LEVELS - 1])
        G[f"e{LEVELS - 1}b"] = act(LEVELS - 1, ch[LEVELS - 1])
        b["r"] = torch.empty((B, H, W), dtype=torch.float32, device=dev)
        scratch = max(nn.wgrad_scratch_bytes(B, res[int(name[1])][0], res[int(name[1])][1], ci, co)
                      for name, ci, co in self.table)
        b["scratch"] = torch.empty(max(scratch, nn.head_scratch_bytes(self.base)), dtype=torch.uint8, device=dev)
        b["ch"] = ch
        self._bufs[key] = b
        return b

    def flipped(self, name: str) -> torch.Tensor:
        ci, co = self.shapes[name]
        if name not in self._flip:
            self._flip[name] = torch.empty((ci, 9, co), dtype=torch.bfloat16, device=self.device)
        nn.conv3x3_flip(self.weight(name), self._flip[name])
        return self._flip[name]

    # -- forward / backward -----------------------------------------------------
    @staticmethod
    def _run(probe, op: str, name: str, fn, ins: Dict, outs: Dict) -> None:
        """Run one layer call; ``probe(stage, op, name, ins, outs)`` (if given)
        sees its operands before ("pre") and after ("post") the call."""
        if probe is not None:
            probe("pre", op, name, ins, outs)
        fn()
        if probe is not None:
            probe("post", op, name, ins, outs)

    def forward(self, x: torch.Tensor, probe=None) -> torch.Tensor:
        """``x [B][H][W][cin]`` bf16 -> ``r [B][H][W]`` float32 (a buffer of the net).
        ``probe``: optional observer of every layer call (see ``_run``)."""
        B, H, W, C = x.shape
        if C != self.cin:
            raise ValueError(f"expected {self.cin} input channels")
        b = self.buffers(B, H, W)
        A = b["act"]
        self._x = x
        run = self._run
        h = x
        for l in range(LEVELS):
            if l > 0:
                xin, yout = A[f"e{l - 1}b"], A[f"in{l}"]
                run(probe, "avgpool2", f"in{l}", lambda: nn.avgpool2(xin, yout), {"x": xin}, {"y": yout})
                h = A[f"in{l}"]
            for name, xin in ((f"e{l}a", h), (f"e{l}b", A[f"e{l}a"])):
                w, bias, y = self.weight(name), self.bias(name), A[name]
                run(probe, "conv", name, lambda: nn.conv3x3(xin, w, bias, y, relu=True),
                    {"x": xin, "w": w, "b": bias}, {"y": y})
        d = A[f"e{LEVELS - 1}b"]
        ch = b["ch"]
        for l in range(LEVELS - 2, -1, -1):
            up = A[f"cat{l}"][..., ch[l]:]
            run(probe, "upsample2", f"cat{l}", lambda: nn.upsample2(d, up), {"x": d}, {"y": up})
            for name, xin in ((f"d{l}a", A[f"cat{l}"]), (f"d{l}b", A[f"d{l}a"])):
                w, bias, y = self.weight(name), self.bias(name), A[name]
                run(probe, "conv", name, lambda: nn.conv3x3(xin, w, bias, y, relu=True),
                    {"x": xin, "w": w, "b": bias}, {"y": y})
            d = A[f"d{l}b"]
        hw, hb, r = self.head_w(), self.head_b(), b["r"]
        run(probe, "head", "head", lambda: nn.head(d, hw, hb, r), {"x": d, "w": hw, "b": hb}, {"r": r})
        self._key = (B, H, W)
        return b["r"]

    def _layer_backward(self, b, name: str, x, dy, dx, mask, probe=None) -> None:
        """Weight / bias gradients of layer ``name`` (input x, pre-activation
        gradient dy) and, if dx is given, the data gradient (masked by the
        ReLU output that fed the layer, if any)."""
        gw, gb = self.grad_views(name)
        self._run(probe, "wgrad", name, lambda: nn.conv3x3_wgrad(x, dy, gw, gb, b["scratch"]),
                  {"x": x, "dy": dy}, {"dw": gw, "db": gb})
        if dx is not None:
            wt = self.flipped(name)
            self._run(probe, "dgrad", name, lambda: nn.conv3x3(dy, wt, None, dx, mask=mask),
                      {"dy": dy, "w": self.weight(name), "mask": mask}, {"dx": dx})

    def backward(self, dr: torch.Tensor, probe=None) -> None:
        """Gradients of ``sum(dr * r)`` for the last forward into ``self.grad``.
        ``probe``: optional observer of every layer call (see ``_run``)."""
        b = self._bufs[self._key]
        A, G, ch = b["act"], b["grad"], b["ch"]
        run = self._run
        hw = self.grad[self.head_off:self.head_off + self.base]
        hb = self.grad[self.head_off + self.base:self.head_off + self.base + 1]
        drc = dr.contiguous()
        run(probe, "head_backward", "head",
            lambda: nn.head_backward(A["d0b"], self.head_w(), drc, G["d0b"], hw, hb, b["scratch"]),
            {"x": A["d0b"], "w": self.head_w(), "dr": drc}, {"dx": G["d0b"], "dw": hw, "db": hb})
        for l in range(LEVELS - 1):
            self._layer_backward(b, f"d{l}b", A[f"d{l}a"], G[f"d{l}b"], G[f"d{l}a"], A[f"d{l}a"], probe)
            self._layer_backward(b, f"d{l}a", A[f"cat{l}"], G[f"d{l}a"], G[f"cat{l}"], A[f"cat{l}"], probe)
            below = f"d{l + 1}b" if l + 1 < LEVELS - 1 else f"e{LEVELS - 1}b"
            dyu, dxu, mu = G[f"cat{l}"][..., ch[l]:], G[below], A[below]
            run(probe, "upsample2_backward", below, lambda: nn.upsample2_backward(dyu, dxu, mask=mu),
                {"dy": dyu, "mask": mu}, {"dx": dxu})
        for l in range(LEVELS - 1, -1, -1):
            self._layer_backward(b, f"e{l}b", A[f"e{l}a"], G[f"e{l}b"], G[f"e{l}a"], A[f"e{l}a"], probe)
            if l > 0:
                self._layer_backward(b, f"e{l}a", A[f"in{l}"], G[f"e{l}a"], G[f"in{l}"], None, probe)
                dyp, dxp, mp = G[f"in{l}"], G[f"e{l - 1}b"], A[f"e{l - 1}b"]
                run(probe, "avgpool2_backward", f"e{l - 1}b",
                    lambda: nn.avgpool2_backward(dyp, dxp, mask=mp, accumulate=True),
                    {"dy": dyp, "mask": mp}, {"dx": dxp})
            else:
                self._layer_backward(b, "e0a", self._x, G["e0a"], None, None, probe)

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> None:
        self.step += 1
        nn.adam(self.w32, self.grad, self.m, self.v, self.wbf, self.step, lr, b1, b2, eps)


# ---------------------------------------------------------------------------
# Training pairs generated by the method itself
# ---------------------------------------------------------------------------
COARSE_N, FINE_N = 128, 512
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_c512_k8.npz")


def pair_phantoms(wl: I.Workload, j: int):
    """Training phantom j: the 256^2 workload's generators (random-field c
    with ellipses, vessel p0) at the workload's size, seeded by (5, 1, j, ...)
    so that no training seed equals a held-out one."""
    n = wl.grid.nx
    c = I.grf_c(n, np.random.default_rng([5, 1, j]), wl.support_radius_px, corr_px=20.0 * n / 256.0)
    p0 = np.stack([I.vessel_p0(n, np.random.default_rng([5, 1, j, k + 1]), wl.support_radius_px)
                   for k in range(wl.K)])
    return c, p0


def simulate(wl: I.Workload, c: np.ndarray, p0: np.ndarray, noise_seed) -> Tuple[torch.Tensor, torch.Tensor]:
    """Noisy sensor data (1 % of each dataset's peak-to-peak) and weights 1/sigma."""
    plan = pat.Plan(wl.grid, wl.K, wl.sensors)
    try:
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
        data = torch.empty(plan.data_shape, dtype=torch.float32, device="cuda")
        ws = plan.workspace(0)
        plan.forward(T(c), T(p0), data, ws, record=False)
        clean = data.cpu().numpy().astype(np.float64)
        del ws
    finally:
        plan.close()
    noisy, sigma = I.add_noise(clean, noise_seed)
    return (torch.from_numpy(noisy.astype(np.float32)).cuda(),
            torch.from_numpy((1.0 / sigma).astype(np.float32)).cuda())


@dataclasses.dataclass
class CoarseResult:
    c: torch.Tensor          # [n][n] sound speed of the coarse level
    p0: torch.Tensor         # [K][n][n]
    g_p0: torch.Tensor       # [K][n][n] gradient of J wrt p0 at the final iterate
    iters: int
    seconds: float
    dx: float


def coarse_level(y_fine: torch.Tensor, dt_fine: float, w: torch.Tensor, K: int, iters: int = 40,
                 n: int = COARSE_N, c_lo: float = 1400.0, c_hi: float = 1600.0) -> CoarseResult:
    """The coarsest multigrid level of Sec. 3.1 (projected L-BFGS from c = the
    middle of the bounds, p0 = 0), returning its iterate and p0 gradient."""
    from . import recon
    t0 = time.perf_counter()
    wl = I.config3_level(n, K=K)
    g = wl.grid
    y = torch.empty((K, g.nt, wl.m), dtype=torch.float32, device="cuda")
    pat.time_interp(y_fine, dt_fine, y, g.dt)
    prob = recon.Problem(wl, y, w, c_lo, c_hi)
    try:
        x0 = torch.zeros(prob.n, dtype=torch.float32, device="cuda")
        x0[prob.K * prob.N:] = 0.5 * (c_lo + c_hi)
        z0 = torch.empty_like(x0)
        pat.mul(x0, prob.inv_scale, z0)
        z, J, hist, nit = recon.projected_lbfgs(prob, z0, iters)
        x = torch.empty_like(z)
        pat.mul(z, prob.scale, x)
        p0, c = prob.split(x)
        out = CoarseResult(c.clone(), p0.clone(), prob.gp0.clone(), nit, 0.0, g.dx)
        torch.cuda.synchronize()
        out.seconds = time.perf_counter() - t0
    finally:
        prob.close()
    return out


def fine_inputs(coarse: CoarseResult, fine: I.Workload) -> Tuple[torch.Tensor, torch.Tensor]:
    """Interpolated coarse c [H][W] and p0 gradients [K][H][W] on the fine grid
    (same physical positions, Sec. 3.1)."""
    g = fine.grid
    K = coarse.p0.shape[0]
    src = torch.cat([coarse.c.reshape(1, *coarse.c.shape), coarse.g_p0]).contiguous()
    out = torch.empty((K + 1, g.ny, g.nx), dtype=torch.float32, device="cuda")
    pat.prolong_phys(src, coarse.dx, out, g.dx)
    return out[0], out[1:]


class LearnedStart:
    """Inference: the fine-level starting sound speed proposed by the network."""

    def __init__(self, net: UNet, fine: I.Workload, c_lo: float = 1400.0, c_hi: float = 1600.0,
                 c_fixed: float = 1500.0):
        self.net, self.fine = net, fine
        g = fine.grid
        self.x = torch.empty((1, g.ny, g.nx, CIN), dtype=torch.bfloat16, device="cuda")
        self.base = torch.empty((g.ny, g.nx), dtype=torch.float32, device="cuda")
        self.scratch = torch.empty(nn.pack_scratch_bytes(), dtype=torch.uint8, device="cuda")
        mask = torch.from_numpy(fine.mask().astype(np.bool_)).cuda()
        self.lo = torch.where(mask, torch.tensor(c_lo, device="cuda"), torch.tensor(c_fixed, device="cuda")).reshape(-1)
        self.hi = torch.where(mask, torch.tensor(c_hi, device="cuda"), torch.tensor(c_fixed, device="cuda")).reshape(-1)

    def __call__(self, c_up: torch.Tensor, g_up: torch.Tensor) -> torch.Tensor:
        nn.pack_input(c_up.contiguous(), g_up.contiguous(), None, 0, C_SHIFT, C_SCALE, self.x, self.base, None,
                      self.scratch)
        r = self.net.forward(self.x)
        c = self.base.reshape(-1).clone()
        pat.project_update(c, r.reshape(-1), -C_SCALE, self.lo, self.hi)   # c = P(base + scale r)
        return c.view(self.fine.grid.ny, self.fine.grid.nx)


def train(net: UNet, coarse_c: torch.Tensor, coarse_g: torch.Tensor, c_true: torch.Tensor, fine: I.Workload,
          coarse_dx: float, epochs: int, batch: int = 4, lr: float = 1e-3, seed: int = 0, log=None,
          symmetries: Sequence[int] = tuple(range(8)), time_budget: Optional[float] = None) -> List[float]:
    """Adam (step size decayed on a cosine from ``lr`` to 0) on the masked
    squared error of the correction (in units of C_SCALE) over pairs (coarse c [n][h][w], summed p0 gradient [n][h][w],
    true fine c [n][H][W]); every pair is used under each symmetry of the
    square in ``symmetries`` (the sensor ring and grids share them)."""
    g = fine.grid
    H, W = g.ny, g.nx
    npairs = coarse_c.shape[0]
    mask = torch.from_numpy(fine.mask().astype(np.uint8)).cuda()
    X = torch.empty((batch, H, W, CIN), dtype=torch.bfloat16, device="cuda")
    base = torch.empty((batch, H, W), dtype=torch.float32, device="cuda")
    target = torch.empty_like(base)
    up = torch.empty((2, H, W), dtype=torch.float32, device="cuda")
    dr = torch.empty_like(base)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    pack_scratch = torch.empty(nn.pack_scratch_bytes(), dtype=torch.uint8, device="cuda")
    mse_scratch = torch.empty(nn.mse_scratch_bytes(), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(seed)
    items = [(j, s) for j in range(npairs) for s in symmetries]
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(items))
        tot, cnt = 0.0, 0
        for start in range(0, len(order) - batch + 1, batch):
            for bi, it in enumerate(order[start:start + batch]):
                j, s = items[it]
                src = torch.stack([coarse_c[j], coarse_g[j]]).contiguous()
                pat.prolong_phys(src, coarse_dx, up, g.dx)
                nn.pack_input(up[0], up[1], c_true[j], s, C_SHIFT, C_SCALE, X[bi:bi + 1], base[bi], target[bi],
                              pack_scratch)
            r = net.forward(X)
            nn.masked_mse(r, target, mask, dr, out, mse_scratch)
            net.backward(dr)
            # cosine decay of the step size over the run (by time if budgeted, else by epochs)
            if time_budget is not None:
                frac = min(1.0, (time.perf_counter() - t0) / time_budget)
            else:
                frac = (ep + start / len(order)) / epochs
            net.adam(lr * 0.5 * (1.0 + np.cos(np.pi * frac)))
            tot += float(out[0].item())
            cnt += 1
            if time_budget is not None and time.perf_counter() - t0 > time_budget:
                break
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}: loss {losses[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
    return losses


def save_weights(net: UNet, path: str, bf16: bool = True) -> None:
    """``.npz`` of the parameters by name; with ``bf16`` the convolution and
    head weights are stored as their bfloat16 bit patterns (uint16): exactly
    what the kernels use, at half the size (biases stay float32)."""
    st = net.state()
    if bf16:
        for k in st:
            if k.endswith(".w"):
                u = st[k].astype(np.float32).view(np.uint32).astype(np.uint64)
                st[k] = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)
    np.savez_compressed(path, base=np.array([net.base]), cin=np.array([net.cin]), **st)


def load_weights(path: str, device: str = "cuda") -> UNet:
    """Network from ``save_weights`` (bfloat16 bit patterns widen exactly to float32)."""
    with np.load(path, allow_pickle=False) as f:
        net = UNet(base=int(f["base"][0]), cin=int(f["cin"][0]), device=device)
        st = {}
        for k in f.files:
            if k in ("base", "cin"):
                continue
            v = f[k]
            st[k] = (v.astype(np.uint32) << 16).view(np.float32) if v.dtype == np.uint16 else v
        net.load(st)
    return net


# ---------------------------------------------------------------------------
# Fine level from a given start; evaluation against plain multigrid
# ---------------------------------------------------------------------------
def relative_error(c: torch.Tensor, c_true: torch.Tensor, mask: torch.Tensor) -> float:
    """Eq. (12) for c over the reconstruction mask, in percent."""
    return 100.0 * float(torch.linalg.vector_norm((c - c_true)[mask]) / torch.linalg.vector_norm(c_true[mask]))


def fine_level(fine: I.Workload, y_fine: torch.Tensor, w: torch.Tensor, c0: torch.Tensor, p00: torch.Tensor,
               c_true: torch.Tensor, iters: int, target: Optional[float] = None, t_origin: Optional[float] = None,
               c_lo: float = 1400.0, c_hi: float = 1600.0):
    """Projected L-BFGS on the fine level from (p0 = p00, c = c0); E_c and wall
    time (from ``t_origin``) after every iteration; stops once E_c <= target."""
    from . import recon
    t_origin = time.perf_counter() if t_origin is None else t_origin
    prob = recon.Problem(fine, y_fine, w, c_lo, c_hi)
    try:
        x0 = torch.cat([p00.reshape(-1), c0.reshape(-1)]).contiguous()
        z0 = torch.empty_like(x0)
        pat.mul(x0, prob.inv_scale, z0)
        pat.project_update(z0, torch.zeros_like(z0), 0.0, prob.lo_z, prob.hi_z)
        mask = prob.mask
        xs = torch.empty_like(z0)

        def c_of(z):
            pat.mul(z, prob.scale, xs)
            return prob.split(xs)[1]

        E = [relative_error(c_of(z0), c_true, mask)]
        T = [time.perf_counter() - t_origin]

        def cb(it, z, J):
            E.append(relative_error(c_of(z), c_true, mask))
            T.append(time.perf_counter() - t_origin)
            return target is not None and E[-1] <= target

        if not (target is not None and E[0] <= target):
            recon.projected_lbfgs(prob, z0, iters, callback=cb)
        torch.cuda.synchronize()
    finally:
        prob.close()
    return E, T


def first_at(E: Sequence[float], T: Sequence[float], target: float):
    for i, (e, t) in enumerate(zip(E, T)):
        if e <= target:
            return i, t
    return None, None


def _hits(E: Sequence[float], T: Sequence[float], targets: Sequence[float], its_before: int, offset: int):
    """Per target: total iterations and seconds at the first E_c <= target."""
    out = {}
    for tg in targets:
        i, t = first_at(E, T, tg)
        out[f"{tg:g}"] = None if i is None else {"iterations": its_before + i + offset, "seconds": round(t, 2)}
    return out


def evaluate_case(net: Optional[UNet], case: int, K: int = 8, coarse_iters: int = 40, fine_iters: int = 20,
                  targets: Sequence[float] = (2.0, 1.0), plain_multigrid: bool = True, log=None,
                  data_grid: int = FINE_N) -> Dict:
    """One held-out phantom (the 256^2 workload's generators at 512^2, seeds
    5000 + case): plain multigrid 128 -> 256 -> 512 against the coarse level
    followed directly by the fine level, started from the plain interpolation
    of the coarse iterate and from the network's proposal.  For each start:
    E_c at the fine start and after every fine iteration, and the iterations
    and wall time (from the start of the run) at which E_c first falls to each
    target; the fine level stops at the smallest target.

    ``data_grid = 768``: the phantom and its data on the finer 768^2 grid
    (``inputs.data_grid_768``) instead of the finest reconstruction grid, and
    E_c measured against the true sound speed interpolated to each level."""
    from . import recon
    fine = I.config3_level(FINE_N, K=K)
    if data_grid == FINE_N:
        c_np, p0_np = I.phantoms(fine, 5, case=case)
        c_true = torch.from_numpy(c_np.astype(np.float32)).cuda()
        y, w = simulate(fine, c_np, p0_np, noise_seed=5000 + case + 500)
        dt = fine.grid.dt
        truth = c_true
    else:
        dw = I.data_grid_768(K=K)
        c_np, p0_np = I.data_grid_phantoms(dw, 5, case=case)
        y, w = simulate(dw, c_np, p0_np, noise_seed=5000 + case + 500)
        dt = dw.grid.dt
        c_data = torch.from_numpy(c_np.astype(np.float32)).cuda().reshape(1, dw.grid.ny, dw.grid.nx)

        def truth(level):
            out = torch.empty((1, level.grid.ny, level.grid.nx), dtype=torch.float32, device="cuda")
            pat.prolong_phys(c_data, dw.grid.dx, out, level.grid.dx)
            return out[0]
        c_true = truth(fine)
    y_fine = y
    if data_grid != FINE_N:   # the fine level's own time grid
        y_fine = torch.empty((K, fine.grid.nt, fine.m), dtype=torch.float32, device="cuda")
        pat.time_interp(y, dt, y_fine, fine.grid.dt)
    res: Dict = {"case": case}
    stop = min(targets) if targets else None
    # coarse level, shared by both starts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    co = coarse_level(y, dt, w, K, iters=coarse_iters)
    c_up, g_up = fine_inputs(co, fine)
    p0_up = torch.empty((K, fine.grid.ny, fine.grid.nx), dtype=torch.float32, device="cuda")
    pat.prolong_phys(co.p0.contiguous(), co.dx, p0_up, fine.grid.dx)
    torch.cuda.synchronize()
    t_coarse = time.perf_counter() - t0
    res["coarse_seconds"] = round(t_coarse, 3)
    res["coarse_iterations"] = co.iters
    starts = {"interpolated": (c_up.clone(), 0.0)}
    if net is not None:
        t1 = time.perf_counter()
        c_net = LearnedStart(net, fine)(c_up, g_up).clone()
        torch.cuda.synchronize()
        res["network_seconds"] = round(time.perf_counter() - t1, 4)
        starts["learned"] = (c_net, time.perf_counter() - t1)
    for name, (c0, extra) in starts.items():
        t_origin = time.perf_counter() - (t_coarse + extra)
        E, T = fine_level(fine, y_fine, w, c0, p0_up, c_true, fine_iters, target=stop, t_origin=t_origin)
        res[name] = {"E_c_start": round(E[0], 3), "E_c_last": round(E[-1], 3), "fine_iterations": len(E) - 1,
                     "E_c": [round(e, 3) for e in E], "t": [round(t, 2) for t in T],
                     "to_target": _hits(E, T, targets, co.iters, 0)}
        if log:
            log(f"case {case} {name}: E_c start {E[0]:.3f} % -> {E[-1]:.3f} % after {len(E) - 1} fine "
                f"iterations; {res[name]['to_target']}")
    if plain_multigrid:
        levels = [I.config3_level(n, K=K) for n in (COARSE_N, 256, FINE_N)]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = recon.multigrid(levels, y, dt, w, truth, iters=coarse_iters, target_Ec=stop)
        total = time.perf_counter() - t2
        fl = out["levels"][-1]
        its_before = sum(lv.iters for lv in out["levels"][:-1])
        T = [fl.t_start + t for t in fl.t]
        res["plain_multigrid"] = {"E_c_last": round(out["E_c"], 3), "seconds_total": round(total, 2),
                                  "E_c": [round(e, 3) for e in fl.E_c], "t": [round(t, 2) for t in T],
                                  "to_target": _hits(fl.E_c, T, targets, its_before, 1)}
        if log:
            log(f"case {case} plain multigrid: final E_c {out['E_c']:.3f} % in {total:.1f} s; "
                f"{res['plain_multigrid']['to_target']}")
    return res


# ---------------------------------------------------------------------------
# Command line: generate pairs, train, evaluate
# ---------------------------------------------------------------------------
def _dataset_sum(g_p0: torch.Tensor) -> torch.Tensor:
    """Sum over the datasets of the p0 gradients (in dataset order)."""
    out = g_p0[0].clone()
    for k in range(1, g_p0.shape[0]):
        pat.axpby(1.0, out, 1.0, g_p0[k], out)
    return out


def generate_pairs(start: int, count: int, K: int = 8, coarse_iters: int = 40, log=print,
                   batch: int = 1) -> Dict[str, np.ndarray]:
    """Training pairs ``start .. start + count - 1``: each phantom's data on the
    fine grid, the 40-iteration coarse level of plain multigrid, its sound
    speed and summed p0 gradient.  ``batch`` > 1 runs that many coarse
    reconstructions in lockstep (``recon.batched_projected_lbfgs``: shared
    launches), with the same results as one at a time."""
    from . import recon
    fine = I.config3_level(FINE_N, K=K)
    coarse = I.config3_level(COARSE_N, K=K)
    m = torch.from_numpy(fine.mask().astype(np.bool_)).cuda()
    cs, gs, ecs, secs = [], [], [], []
    for g0 in range(start, start + count, batch):
        group = list(range(g0, min(g0 + batch, start + count)))
        t0 = time.perf_counter()
        truths, probs, z0s = [], [], []
        for j in group:
            c_np, p0_np = pair_phantoms(fine, j)
            y, w = simulate(fine, c_np, p0_np, noise_seed=[5, 1, j, 500])
            truths.append(c_np)
            if batch == 1:
                co = coarse_level(y, fine.grid.dt, w, K, iters=coarse_iters)
                results = [(co.c, co.g_p0, co.iters, co.dx)]
                break
            g = coarse.grid
            yc = torch.empty((K, g.nt, coarse.m), dtype=torch.float32, device="cuda")
            pat.time_interp(y, fine.grid.dt, yc, g.dt)
            del y
            prob = recon.Problem(coarse, yc, w, 1400.0, 1600.0)
            x0 = torch.zeros(prob.n, dtype=torch.float32, device="cuda")
            x0[prob.K * prob.N:] = 1500.0
            z0 = torch.empty_like(x0)
            pat.mul(x0, prob.inv_scale, z0)
            probs.append(prob)
            z0s.append(z0)
        if batch > 1:
            out = recon.batched_projected_lbfgs(probs, z0s, coarse_iters)
            results = []
            for prob, (z, J, hist, nit) in zip(probs, out):
                x = torch.empty_like(z)
                pat.mul(z, prob.scale, x)
                results.append((prob.split(x)[1].clone(), prob.gp0.clone(), nit, coarse.grid.dx))
                prob.close()
        torch.cuda.synchronize()
        dt_each = (time.perf_counter() - t0) / len(group)
        for j, c_np, (c, gp0, nit, dx) in zip(group, truths, results):
            cs.append(c.cpu().numpy())
            gs.append(_dataset_sum(gp0).cpu().numpy())
            co = CoarseResult(c, gp0, gp0, nit, 0.0, dx)
            c_up, _ = fine_inputs(co, fine)
            ecs.append(relative_error(c_up, torch.from_numpy(c_np.astype(np.float32)).cuda(), m))
            secs.append(dt_each)
            if log:
                log(f"pair {j}: coarse iterations {nit}, interpolated E_c {ecs[-1]:.3f} %, {dt_each:.2f} s")
    return {"index": np.arange(start, start + count), "c": np.stack(cs).astype(np.float32),
            "gsum": np.stack(gs).astype(np.float32), "E_c_interp": np.array(ecs), "seconds": np.array(secs)}


def truth_for_pairs(index: Sequence[int], K: int = 8) -> np.ndarray:
    """True 512^2 sound speeds of training pairs (the sound-speed draw of
    ``pair_phantoms`` alone)."""
    fine = I.config3_level(FINE_N, K=K)
    n = fine.grid.nx
    return np.stack([I.grf_c(n, np.random.default_rng([5, 1, int(j)]), fine.support_radius_px,
                             corr_px=20.0 * n / 256.0) for j in index]).astype(np.float32)


def network_flops(net: UNet, B: int, H: int, W: int) -> Tuple[float, float]:
    """Multiply-add flops (2 per product) of the 3x3 convolutions: forward, and
    forward + both backward contractions (data gradient skipped for the first
    layer, whose input needs none)."""
    fwd = bwd = 0.0
    for name, ci, co in net.table:
        lvl = int(name[1])
        f = 2.0 * B * (H >> lvl) * (W >> lvl) * 9 * ci * co
        fwd += f
        bwd += f if name == "e0a" else 2.0 * f
    return fwd, fwd + bwd


def network_roofline_ms(net: UNet, B: int, H: int, W: int, mfma_tflops: float = 2500.0,
                        hbm_gbs: float = 8000.0) -> float:
    """Lower bound of the forward convolutions: per layer the larger of its
    flops at the dense bf16 MFMA peak and its bf16 input + output + weight
    bytes at the HBM peak, summed over the layers (milliseconds)."""
    t = 0.0
    for name, ci, co in net.table:
        lvl = int(name[1])
        P = B * (H >> lvl) * (W >> lvl)
        f = 2.0 * P * 9 * ci * co
        by = 2.0 * (P * (ci + co) + co * 9 * ci)
        t += max(f / (mfma_tflops * 1e12), by / (hbm_gbs * 1e9))
    return 1e3 * t


def time_network(B: int = 4, steps: int = 5, H: int = FINE_N, W: int = FINE_N) -> Dict:
    """Average wall time of the forward pass and of one training step (forward,
    loss, backward, Adam) on random inputs, and the convolution flop rates."""
    net = load_weights(DEFAULT_WEIGHTS) if os.path.exists(DEFAULT_WEIGHTS) else UNet(base=32)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((B, H, W, CIN), device="cuda", generator=g).to(torch.bfloat16)
    t = torch.randn((B, H, W), device="cuda", generator=g)
    mask = torch.ones((H, W), dtype=torch.uint8, device="cuda")
    dr = torch.empty_like(t)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    sc = torch.empty(nn.mse_scratch_bytes(), dtype=torch.uint8, device="cuda")

    def step():
        r = net.forward(x)
        nn.masked_mse(r, t, mask, dr, out, sc)
        net.backward(dr)
        net.adam(1e-5)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.forward(x)
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / steps
    ff, ft = network_flops(net, B, H, W)
    roof = network_roofline_ms(net, B, H, W)
    return {"batch": B, "size": [H, W], "forward_ms": round(1e3 * tf, 3), "train_step_ms": round(1e3 * ts, 3),
            "forward_roofline_ms": round(roof, 4), "forward_roofline_frac": round(roof / (1e3 * tf), 3),
            "forward_conv_TFLOPs": round(ff / tf / 1e12, 1), "train_conv_TFLOPs": round(ft / ts / 1e12, 1),
            "forward_GFLOP": round(ff / 1e9, 2), "train_GFLOP": round(ft / 1e9, 2)}


RUNS = (("plain_multigrid", "plain multigrid 128 -> 256 -> 512"),
        ("interpolated", "coarse level, then 512^2 from the interpolated coarse iterate"),
        ("learned", "coarse level, then 512^2 from the network's proposal"))


def summarize(rows: Sequence[Dict], targets: Sequence[float] = (2.0, 1.0)) -> Tuple[Dict, str]:
    """Per start (plain multigrid, interpolated, learned) over the evaluated
    cases: fine-level start E_c (mean, median), and per target the cases that
    reach it with the mean and median wall time and iterations to it.  Returns
    the figures and a markdown table of them."""
    out: Dict = {"cases": len(rows)}
    lines = ["| run | fine-start E_c mean / median | " + " | ".join(
        f"reaches {tg:g} % | s to {tg:g} % mean / median | iterations to {tg:g} % mean" for tg in targets) + " |",
        "|---|---:|" + "---:|---:|---:|" * len(targets)]
    for run, label in RUNS:
        have = [r for r in rows if run in r]
        if not have:
            continue
        if run == "plain_multigrid":
            starts = [r[run]["E_c"][0] for r in have if r[run]["E_c"]]
        else:
            starts = [r[run]["E_c_start"] for r in have]
        fig = {"E_c_start_mean": round(float(np.mean(starts)), 3), "E_c_start_median": round(float(np.median(starts)), 3)}
        cells = [f"{fig['E_c_start_mean']:.2f} % / {fig['E_c_start_median']:.2f} %"]
        for tg in targets:
            hits = [r[run]["to_target"][f"{tg:g}"] for r in have]
            ok = [h for h in hits if h is not None]
            sec = [h["seconds"] for h in ok]
            its = [h["iterations"] for h in ok]
            fig[f"{tg:g}"] = {"reached": len(ok), "of": len(have),
                              "seconds_mean": round(float(np.mean(sec)), 2) if ok else None,
                              "seconds_median": round(float(np.median(sec)), 2) if ok else None,
                              "iterations_mean": round(float(np.mean(its)), 1) if ok else None}
            f = fig[f"{tg:g}"]
            cells += [f"{len(ok)}/{len(have)}",
                      f"{f['seconds_mean']:.2f} / {f['seconds_median']:.2f}" if ok else "-",
                      f"{f['iterations_mean']:.1f}" if ok else "-"]
        out[run] = fig
        lines.append(f"| {label} | " + " | ".join(cells) + " |")
    return out, "\n".join(lines)


def main(argv=None) -> int:
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("gen", help="generate training pairs with the plain method")
    g.add_argument("--start", type=int, default=0)
    g.add_argument("--count", type=int, default=8)
    g.add_argument("--out", required=True)
    g.add_argument("--batch", type=int, default=1, help="coarse reconstructions run in lockstep")
    t = sub.add_parser("train", help="train the network on generated pairs")
    t.add_argument("--pairs", nargs="+", required=True)
    t.add_argument("--epochs", type=int, default=10)
    t.add_argument("--batch", type=int, default=4)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--minutes", type=float, default=None, help="stop after this much training time")
    t.add_argument("--holdout", type=int, default=0, help="pairs kept out of training for a validation loss")
    t.add_argument("--out", required=True)
    tm = sub.add_parser("time", help="time the network's forward pass and training step at 512^2")
    tm.add_argument("--batch", type=int, default=4)
    tm.add_argument("--steps", type=int, default=5)
    e = sub.add_parser("eval", help="held-out phantoms: learned start vs plain multigrid")
    e.add_argument("--weights", default=None)
    e.add_argument("--cases", type=int, nargs="+", default=[0, 1])
    e.add_argument("--fine-iters", type=int, default=20)
    e.add_argument("--no-multigrid", action="store_true")
    e.add_argument("--data-grid", type=int, default=FINE_N, choices=(FINE_N, 768),
                   help="grid the phantom's data are simulated on (768: finer than the reconstruction grid)")
    e.add_argument("--out", default=None)
    sm = sub.add_parser("summary", help="table of the runs in evaluation files written by eval --out")
    sm.add_argument("files", nargs="+")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    if a.cmd == "gen":
        d = generate_pairs(a.start, a.count, log=log, batch=a.batch)
        np.savez(a.out, **d)
        return 0
    if a.cmd == "train":
        parts = [np.load(p, allow_pickle=False) for p in a.pairs]
        index = np.concatenate([p["index"] for p in parts])
        cc = np.concatenate([p["c"] for p in parts])
        gg = np.concatenate([p["gsum"] for p in parts])
        ntr = len(index) - a.holdout
        log(f"{len(index)} pairs ({ntr} for training), generating the true 512^2 sound speeds")
        truth = truth_for_pairs(index)
        fine = I.config3_level(FINE_N, K=8)
        coarse_dx = I.config3_level(COARSE_N, K=8).grid.dx
        T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
        net = UNet(base=32, seed=0)
        t0 = time.perf_counter()
        losses = train(net, T(cc[:ntr]), T(gg[:ntr]), T(truth[:ntr]), fine, coarse_dx, a.epochs, batch=a.batch,
                       lr=a.lr, log=log, time_budget=None if a.minutes is None else 60.0 * a.minutes)
        torch.cuda.synchronize()
        log(f"trained {net.step} steps in {time.perf_counter() - t0:.1f} s")
        save_weights(net, a.out)
        if a.holdout:
            ls = LearnedStart(net, fine)
            mask = torch.from_numpy(fine.mask().astype(np.bool_)).cuda()
            e0, e1 = [], []
            for j in range(ntr, len(index)):
                c_up = torch.empty((2, fine.grid.ny, fine.grid.nx), dtype=torch.float32, device="cuda")
                pat.prolong_phys(T(np.stack([cc[j], gg[j]])), coarse_dx, c_up, fine.grid.dx)
                ct = T(truth[j])
                e0.append(relative_error(c_up[0], ct, mask))
                e1.append(relative_error(ls(c_up[0], c_up[1:2]), ct, mask))
            log(f"held-out pairs: E_c interpolated {np.mean(e0):.3f} %, learned {np.mean(e1):.3f} %")
        return 0
    if a.cmd == "time":
        print(json.dumps(time_network(a.batch, a.steps)), flush=True)
        return 0
    if a.cmd == "summary":
        rows = []
        for f in a.files:
            with open(f) as fh:
                rows += json.load(fh)
        fig, table = summarize(rows)
        print(json.dumps(fig, indent=1))
        print(table)
        return 0
    if a.cmd == "eval":
        net = load_weights(a.weights) if a.weights else None
        rows = [evaluate_case(net, c, fine_iters=a.fine_iters, plain_multigrid=not a.no_multigrid, log=log,
                              data_grid=a.data_grid) for c in a.cases]
        if a.out:
            with open(a.out, "w") as f:
                json.dump(rows, f, indent=1)
        return 0
    return 1


if __name__ == "__main__":
    raise SystemExit(main())
