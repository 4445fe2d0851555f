"""GPU: every kernel of the surrogate, element by element, at the training size and
at a ragged one.

One forward and backward pass of the network at 256^2 (batch 2) and at 40^2 (batch
3: every map ends in partial tiles) runs with the library's trace on, so that the BF16 tensors each kernel read and wrote can be
read back (sur_read).  Each kernel is then recomputed in FP64 by the oracle from
exactly the BF16 operands that kernel used on the GPU (its input activation or
output gradient as stored, the BF16-rounded weights), so the only differences left
are the kernel's own FP32 accumulation and its output rounding.  Per element:

    |gpu - ref| <= (1 + 2^-8) (K + 2) 2^-24 S + 2^-8 |ref|   (BF16 output)
    |gpu - ref| <= (K + 2) 2^-24 S                           (FP32 output)

with 2^-24 and 2^-8 the unit roundoffs of FP32 and of BF16 (8-bit significand),
S the same sum over absolute values (sum |w| |x| + |b|) and K the number of
FP32 additions behind the element: 9 c_in (padded) for a convolution, 9 c_out
(padded) for its input gradient, a workgroup's run of pixels plus the runs' atomic
additions for a weight gradient, 3 for pooling, and for the upsampling gradient (summed from
the FP32 input gradient inside the kernel that computes it) that input gradient's plus 3.  Copies (upsampling
into the concatenations) must be exact.  A misplaced tile, halo column, channel
pair or pixel run changes elements by the size of the values themselves, far
beyond these bounds.
"""
import numpy as np
import pytest

from oracle import surrogate as S

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_1611_00907_amd.lbm")

# the training size, and a size whose maps (40, 20, 10, 5) end in ragged tiles of every
# convolution kernel and take the gather weight-gradient kernel (widths not a multiple of 32)
SHAPES = [(256, 2), (40, 3)]
U32 = 2.0 ** -24
U16 = 2.0 ** -8          # unit roundoff of BF16 (8-bit significand, round to nearest)


def wgrad_terms(n, h, w, cin, cout):
    """FP32 additions behind one weight-gradient element in the library's schedule.
    Layers of 32-128 output channels (the LDS kernel): runs of at least 8 tiles of
    4 x 32 pixels, at most about 512 workgroups over all 32-channel input blocks, one
    atomic addition per run; counted as every pixel of a run plus the runs.  Maps
    whose width is not a multiple of 32: the gather kernel's pixel runs.  The one-output-channel layer:
    runs of 256-8192 pixels in 16 groups, the reduction across the block, one atomic
    addition per run."""
    px = n * h * w
    if cout == 1:
        run = min(max((px // 2048 + 15) // 16 * 16, 256), 8192)
        return run + 16 + (px + run - 1) // run
    if not (cout % 32 == 0 and cout <= 128 and w % 32 == 0 and h % 4 == 0 and cin % 8 == 0):
        # the gather kernel: pixel runs of 512-8192 sized for about 16384 waves
        blocks = 9 * ((cout + 31) // 32) * ((cin + 31) // 32)
        run = min(max(px * blocks // 16384, 512), 8192) // 32 * 32
        return run + 16 + (px + run - 1) // run
    tiles = n * (h // 4) * (w // 32)
    runs = max(min(512 // ((cin + 31) // 32), (tiles + 7) // 8), 1)
    per_run = (tiles + runs - 1) // runs
    runs = (tiles + per_run - 1) // per_run
    return 128 * per_run + 16 + runs


def bf16(a):
    """Round to bfloat16, nearest even, returned as float64 (what the library's
    FP32 -> BF16 conversion does)."""
    bits = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def nchw(t):
    return np.ascontiguousarray(t.transpose(0, 3, 1, 2), dtype=np.float64)


@pytest.fixture(scope="module", params=SHAPES, ids=["%dx%d" % s for s in SHAPES])
def run(request):
    SIZE, BATCH = request.param
    r = np.random.default_rng(21)
    params = S.init_params(17)
    params = {k: (w, r.normal(0, 0.05, b.shape)) for k, (w, b) in params.items()}
    x = r.normal(size=(BATCH, S.IN_CHANNELS, SIZE, SIZE)).astype(np.float32)
    t = r.normal(size=(BATCH, SIZE, SIZE)).astype(np.float32)
    net = lbm.Surrogate(SIZE, max_batch=BATCH)
    flat = lbm.Surrogate.flatten(params)
    net.set_params(flat)
    net.trace(True)
    g, loss = net.gradients(x, t)
    names = ["x0", "e0a", "c0", "p0", "e1a", "c1", "p1", "e2a", "c2", "p2", "e3a", "e3", "d2a", "d2", "d1a",
             "d1", "d0a", "d0", "y", "dc0", "dc1", "dc2", "dp_e3a", "dp_e2a", "dp_e1a"]
    names += ["dz_" + name for name, _, _ in lbm.Surrogate.LAYERS]
    T = {k: nchw(net.read(k)) for k in names}
    net.close()
    master = lbm.Surrogate.unflatten(flat.astype(np.float64))          # the FP32 master copy
    W = {k: (bf16(w), b) for k, (w, b) in master.items()}              # what the kernels multiply
    grads = lbm.Surrogate.unflatten(g.astype(np.float64))
    return {"T": T, "W": W, "grads": grads, "loss": loss, "x": x, "t": t}


def check(label, got, ref, scale, K, bf16_out):
    gamma = (K + 2) * U32
    bound = gamma * scale * (1 + U16) + (U16 * np.abs(ref) if bf16_out else 0.0) + 1e-38
    err = np.abs(got - ref)
    worst = float(np.max(err / bound))
    print("%-28s max err/bound %.3g  (max |ref| %.3g)" % (label, worst, float(np.max(np.abs(ref)))))
    assert got.shape == ref.shape, label
    assert worst <= 1.0, (label, worst, np.unravel_index(np.argmax(err / bound), err.shape))


LAYER_IO = [  # layer, input tensor (channel slice), output tensor (channel slice)
    ("e0a", ("x0", None), ("e0a", None)), ("e0b", ("e0a", None), ("c0", (64, 96))),
    ("e1a", ("p0", None), ("e1a", None)), ("e1b", ("e1a", None), ("c1", (96, 160))),
    ("e2a", ("p1", None), ("e2a", None)), ("e2b", ("e2a", None), ("c2", (128, 224))),
    ("e3a", ("p2", None), ("e3a", None)), ("e3b", ("e3a", None), ("e3", None)),
    ("d2a", ("c2", None), ("d2a", None)), ("d2b", ("d2a", None), ("d2", None)),
    ("d1a", ("c1", None), ("d1a", None)), ("d1b", ("d1a", None), ("d1", None)),
    ("d0a", ("c0", None), ("d0a", None)), ("d0b", ("d0a", None), ("d0", None)),
    ("out", ("d0", None), ("y", None)),
]


def _sl(T, spec):
    name, ch = spec
    a = T[name]
    return a if ch is None else a[:, ch[0]:ch[1]]


def _pad(c, m):
    return (c + m - 1) // m * m


@pytest.mark.parametrize("layer,src,dst", LAYER_IO, ids=[io[0] for io in LAYER_IO])
def test_forward_convolution(run, layer, src, dst):
    T, (w, b) = run["T"], run["W"][layer]
    x = _sl(T, src)
    ref = S.conv3x3(x, w, b)
    scale = S.conv3x3(np.abs(x), np.abs(w), np.abs(b))
    if layer != "out":
        ref = S.relu(ref)
    check("forward " + layer, _sl(T, dst), ref, scale, 9 * _pad(w.shape[1], 32), bf16_out=layer != "out")


@pytest.mark.parametrize("layer,src", [(io[0], io[1]) for io in LAYER_IO], ids=[io[0] for io in LAYER_IO])
def test_weight_and_bias_gradients(run, layer, src):
    T, grads = run["T"], run["grads"]
    x = _sl(T, src)
    dz = T["dz_" + layer]
    if layer == "out":
        dz = dz[:, :1]
    dw, db = S.conv3x3_grad_weight(x, dz)
    sw, sb = S.conv3x3_grad_weight(np.abs(x), np.abs(dz))
    K = wgrad_terms(x.shape[0], x.shape[2], x.shape[3], x.shape[1], dz.shape[1])
    check("weight gradient " + layer, grads[layer][0], dw, sw, K, bf16_out=False)
    check("bias gradient " + layer, grads[layer][1], db, sb, K, bf16_out=False)


# (layer whose input gradient is taken, its output gradient dz, the ReLU mask of its
#  input, the GPU tensor the masked BF16 result went to)
MASKED_BACK = [("out", "dz_out", "d0", "dz_d0b"), ("d0b", "dz_d0b", "d0a", "dz_d0a"),
               ("d1b", "dz_d1b", "d1a", "dz_d1a"), ("d2b", "dz_d2b", "d2a", "dz_d2a"),
               ("e3b", "dz_e3b", "e3a", "dz_e3a"), ("e2b", "dz_e2b", "e2a", "dz_e2a"),
               ("e1b", "dz_e1b", "e1a", "dz_e1a"), ("e0b", "dz_e0b", "e0a", "dz_e0a")]


@pytest.mark.parametrize("layer,dzn,maskn,dst", MASKED_BACK, ids=[m[0] for m in MASKED_BACK])
def test_input_gradient_through_relu(run, layer, dzn, maskn, dst):
    T, (w, _) = run["T"], run["W"][layer]
    dz = T[dzn][:, :w.shape[0]]
    keep = T[maskn] > 0
    ref = S.conv3x3_grad_input(dz, w) * keep
    scale = S.conv3x3_grad_input(np.abs(dz), np.abs(w)) * keep
    check("input gradient " + layer, T[dst], ref, scale, 9 * _pad(w.shape[0], 32), bf16_out=True)


# input gradients kept in FP32: the concatenations' and the pooled branches'.  A
# decoder's input gradient stores only its skip share: the kernel that computes it
# folds the upsampled share into the upsampling gradient at once (checked below from
# the oracle's own input gradient).
F32_BACK = [("d0a", "dz_d0a", "dc0", (64, 96)), ("d1a", "dz_d1a", "dc1", (96, 160)), ("d2a", "dz_d2a", "dc2", (128, 224)),
            ("e3a", "dz_e3a", "dp_e3a", None), ("e2a", "dz_e2a", "dp_e2a", None), ("e1a", "dz_e1a", "dp_e1a", None)]


@pytest.mark.parametrize("layer,dzn,dst,ch", F32_BACK, ids=[m[0] for m in F32_BACK])
def test_input_gradient_fp32(run, layer, dzn, dst, ch):
    T, (w, _) = run["T"], run["W"][layer]
    dz = T[dzn]
    ref = S.conv3x3_grad_input(dz, w)
    scale = S.conv3x3_grad_input(np.abs(dz), np.abs(w))
    got = T[dst]
    if ch is not None:
        got, ref, scale = got[:, ch[0]:ch[1]], ref[:, ch[0]:ch[1]], scale[:, ch[0]:ch[1]]
    check("input gradient " + layer, got, ref, scale, 9 * _pad(w.shape[0], 32), bf16_out=False)


def test_pooling_and_upsampling(run):
    """Average pooling of the skip halves (BF16 sums of four, rounded once) and the
    nearest upsampling copies into the concatenations (exact)."""
    T = run["T"]
    for src, dst in ((("c0", (64, 96)), "p0"), (("c1", (96, 160)), "p1"), (("c2", (128, 224)), "p2")):
        a = _sl(T, src)
        check("avgpool " + dst, T[dst], S.avgpool2(a), S.avgpool2(np.abs(a)), 3, bf16_out=True)
    for src, (dst, ch) in (("d1", ("c0", 64)), ("d2", ("c1", 96)), ("e3", ("c2", 128))):
        assert np.array_equal(T[dst][:, :ch], S.upsample2(T[src])), "upsample " + src


UP_GRAD = [("d0a", "dz_d0a", 64, "d1", "dz_d1b"), ("d1a", "dz_d1a", 96, "d2", "dz_d2b"),
           ("d2a", "dz_d2a", 128, "e3", "dz_e3b")]


@pytest.mark.parametrize("layer,dzn,ch,act,dst", UP_GRAD, ids=[u[4] for u in UP_GRAD])
def test_upsampling_gradient(run, layer, dzn, ch, act, dst):
    """The upsampled share of a decoder's FP32 input gradient summed over 2 x 2 blocks
    and masked, from the oracle's input gradient of the stored BF16 operands: the
    convolution's additions plus 3."""
    T, (w, _) = run["T"], run["W"][layer]
    dz = T[dzn]
    keep = T[act] > 0
    ref = S.upsample2_grad(S.conv3x3_grad_input(dz, w)[:, :ch]) * keep
    scale = S.upsample2_grad(S.conv3x3_grad_input(np.abs(dz), np.abs(w))[:, :ch]) * keep
    check("upsampling gradient " + dst, T[dst], ref, scale, 9 * _pad(w.shape[0], 32) + 3, bf16_out=True)


SKIP_GRAD = [("dc2", (128, 224), "dp_e3a", ("c2", (128, 224)), "dz_e2b"),
             ("dc1", (96, 160), "dp_e2a", ("c1", (96, 160)), "dz_e1b"),
             ("dc0", (64, 96), "dp_e1a", ("c0", (64, 96)), "dz_e0b")]


@pytest.mark.parametrize("dcat,ch,dp,act,dst", SKIP_GRAD, ids=[s[4] for s in SKIP_GRAD])
def test_skip_gradient(run, dcat, ch, dp, act, dst):
    """The skip half of a concatenation's gradient plus the pooling gradient of the
    level below, through the ReLU of the skip activation."""
    T = run["T"]
    d = T[dcat][:, ch[0]:ch[1]]
    keep = _sl(T, act) > 0
    ref = (d + S.avgpool2_grad(T[dp])) * keep
    scale = (np.abs(d) + S.avgpool2_grad(np.abs(T[dp]))) * keep
    check("skip gradient " + dst, T[dst], ref, scale, 2, bf16_out=True)


def test_loss_and_output_gradient(run):
    """MSE on the GPU's own prediction: dY = 2 (y - t) / count in BF16, channel 0 only."""
    T = run["T"]
    y = T["y"][:, 0]
    t = run["t"].astype(np.float64)
    d = y - t
    assert run["loss"] == pytest.approx(float((d * d).mean()), rel=1e-6)
    ref = 2.0 * d / d.size
    check("output gradient", T["dz_out"][:, 0], ref, 2.0 * (np.abs(y) + np.abs(t)) / d.size, 2, bf16_out=True)
    assert not np.any(T["dz_out"][:, 1:])


def test_packed_input(run):
    T = run["T"]
    assert np.array_equal(T["x0"][:, :4], bf16(run["x"]))
    assert not np.any(T["x0"][:, 4:])
