"""Layer-by-layer replay of the learned-start network at its full size.

One forward + backward of the U-Net (base 32, one 512 x 512 image, the fine
level of the learned start) runs on the GPU with a probe on every layer call.
Each call's operands are read back exactly as the GPU holds them (bf16
activations and gradients, bf16 weights, float32 biases), the oracle layer
(oracle/unet.py) is applied to those same values in float64, and the GPU
output is compared element by element within the layer's arithmetic bound:

* bf16 results (convolutions, data gradients, pooling, adjoints of pooling and
  upsampling, the head's data gradient): ``(2^-8 + 2^-22) |ref| + 1e-5 S``
  (the unit roundoff 2^-8 of bf16's 8-bit significand for the rounding of
  the result, a float32 rounding before it, and the float32 accumulation,
  ``S`` the same sum over absolute values);
* float32 results (weight and bias gradients, the head): ``2^-23 |ref| + 1e-5 S``;
* the upsampling copy: exact.

Replaying each layer on the GPU's own inputs removes the cascade through which
one bf16 rounding that lands on the other side of a boundary moves every
later layer, so a wrong layer anywhere in the chain fails its own bound.  Run
with random weights and with the trained weights on a smooth input.
"""
import os

import numpy as np
import pytest

from oracle import unet as U
from tests.gpu_helpers import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_08482_amd import inputs as I  # noqa: E402
from paper_2505_08482_amd import learned, nn  # noqa: E402

BF16_REL = 2.0 ** -8 + 2.0 ** -22
F32_REL = 2.0 ** -23
ACC = 1e-5


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def ratio(got, ref, S, rel):
    """Largest error relative to its bound (<= 1 passes)."""
    bound = rel * np.abs(ref) + ACC * S + 1e-30
    return float(np.max(np.abs(got - ref) / bound))


class Replay:
    """Probe: checks every layer call against the oracle on the call's own operands."""

    def __init__(self):
        self.worst = {}
        self.prior = None
        self.count = 0

    def _record(self, key, r):
        self.worst[key] = max(self.worst.get(key, 0.0), r)

    def __call__(self, stage, op, name, ins, outs):
        torch.cuda.synchronize()
        if stage == "pre":
            if op == "avgpool2_backward":        # accumulates into its output
                self.prior = host(outs["dx"])
            return
        self.count += 1
        a = {k: host(v) for k, v in ins.items() if v is not None}
        key = f"{op}:{name}"
        if op == "conv":
            ref = U.relu(U.conv3x3(a["x"], a["w"], a["b"]))
            S = U.conv3x3(np.abs(a["x"]), np.abs(a["w"]), np.abs(a["b"]))
            self._record(key, ratio(host(outs["y"]), ref, S, BF16_REL))
        elif op == "dgrad":
            ref = U.conv3x3_data_gradient(a["w"], a["dy"])
            S = U.conv3x3_data_gradient(np.abs(a["w"]), np.abs(a["dy"]))
            if "mask" in a:
                ref = ref * (a["mask"] > 0)
            self._record(key, ratio(host(outs["dx"]), ref, S, BF16_REL))
        elif op == "wgrad":
            dw, db = U.conv3x3_weight_gradient(a["x"], a["dy"])
            Sw, Sb = U.conv3x3_weight_gradient(np.abs(a["x"]), np.abs(a["dy"]))
            got_w = host(outs["dw"]).reshape(dw.shape)
            self._record(key, max(ratio(got_w, dw, Sw, F32_REL), ratio(host(outs["db"]), db, Sb, F32_REL)))
        elif op == "avgpool2":
            ref = U.avgpool2(a["x"])
            self._record(key, ratio(host(outs["y"]), ref, U.avgpool2(np.abs(a["x"])), BF16_REL))
        elif op == "upsample2":
            got = host(outs["y"])
            self._record(key, 0.0 if np.array_equal(got, U.upsample2(a["x"])) else np.inf)
        elif op == "upsample2_backward":
            ref = U.upsample2_backward(a["dy"]) * (a["mask"] > 0)
            S = U.upsample2_backward(np.abs(a["dy"]))
            self._record(key, ratio(host(outs["dx"]), ref, S, BF16_REL))
        elif op == "avgpool2_backward":
            ref = (self.prior + U.avgpool2_backward(a["dy"])) * (a["mask"] > 0)
            S = np.abs(self.prior) + U.avgpool2_backward(np.abs(a["dy"]))
            self._record(key, ratio(host(outs["dx"]), ref, S, BF16_REL))
        elif op == "head":
            ref = U.head(a["x"], a["w"], float(a["b"][0]))
            S = U.head(np.abs(a["x"]), np.abs(a["w"]), abs(float(a["b"][0])))
            self._record(key, ratio(host(outs["r"]), ref, S, F32_REL))
        elif op == "head_backward":
            dx, dw, db = U.head_backward(a["x"], a["w"], a["dr"])
            dx = dx * (a["x"] > 0)
            _, Sw, Sb = U.head_backward(np.abs(a["x"]), np.abs(a["w"]), np.abs(a["dr"]))
            r = max(ratio(host(outs["dx"]), dx, np.abs(dx), BF16_REL),
                    ratio(host(outs["dw"]), dw, Sw, F32_REL),
                    ratio(host(outs["db"]), np.array([db]), np.array([Sb]), F32_REL))
            self._record(key, r)
        else:
            raise AssertionError(f"unknown layer call {op}")


def _smooth_input(n, seed):
    """A sound-speed-like and a gradient-like channel (the learned start's two
    inputs), both smooth random fields, plus the six zero channels."""
    wl = I.config2(n=n, K=1, nt=2)
    c, _ = I.phantoms(wl, 5, case=seed)
    rng = np.random.default_rng(seed)
    g = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal((n, n))) *
                             np.exp(-0.5 * 16.0 ** 2 * (np.fft.fftfreq(n)[:, None] ** 2 +
                                                         np.fft.fftfreq(n)[None, :] ** 2) * (2 * np.pi) ** 2)))
    g = g / np.abs(g).max()
    x = np.zeros((1, n, n, learned.CIN))
    x[0, :, :, 0] = (c - learned.C_SHIFT) / learned.C_SCALE
    x[0, :, :, 1] = g
    return x


@pytest.mark.parametrize("weights", ["random", "trained"])
def test_layer_replay_full_size(weights):
    n = 512
    announce(f"nn layer replay 1x{n}x{n} base 32, {weights} weights")
    if weights == "trained":
        if not os.path.exists(learned.DEFAULT_WEIGHTS):
            pytest.skip("no trained weights")
        net = learned.load_weights(learned.DEFAULT_WEIGHTS)
        x_np = _smooth_input(n, 3)
    else:
        net = learned.UNet(base=32, seed=11)
        rng = np.random.default_rng(12)
        p = U.init_params(net.cin, 32, seed=11)
        for k in list(p):
            if k.endswith(".b"):
                p[k] = 0.05 * rng.standard_normal(p[k].shape)
        p["head.w"] = rng.standard_normal(32) / np.sqrt(32.0)
        p["head.b"] = np.array([0.1])
        net.load(p)
        x_np = np.concatenate([rng.standard_normal((1, n, n, 2)), np.zeros((1, n, n, 6))], axis=-1)
    x = torch.from_numpy(x_np.astype(np.float32)).to(torch.bfloat16).cuda()
    probe = Replay()
    r = net.forward(x, probe=probe)
    rng = np.random.default_rng(13)
    t = torch.from_numpy(rng.standard_normal((1, n, n)).astype(np.float32) * 0.1).cuda()
    mask = torch.from_numpy(I.mask_disc(n, 190.0).astype(np.uint8)).cuda()
    dr = torch.empty_like(r)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    nn.masked_mse(r, t, mask, dr, out, torch.empty(nn.mse_scratch_bytes(), dtype=torch.uint8, device="cuda"))
    net.backward(dr, probe=probe)
    torch.cuda.synchronize()
    worst = max(probe.worst, key=probe.worst.get)
    print(f"[nn replay] {weights}: {probe.count} layer calls, worst {worst} at {probe.worst[worst]:.3f} of its "
          f"bound; " + ", ".join(f"{k} {v:.3f}" for k, v in sorted(probe.worst.items())), flush=True)
    # 14 convolutions, 3 poolings, 3 upsamplings, the head; then the head's
    # backward, 14 weight gradients, 13 data gradients, 3 + 3 pooling adjoints
    assert probe.count == 21 + 34
    assert probe.worst[worst] <= 1.0, (worst, probe.worst[worst])
