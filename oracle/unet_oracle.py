"""FP64 CPU oracle of the learned Poisson part (test infrastructure only).

A small U-Net maps the volume-weighted Poisson right-hand side b (the node
equation of Eq. 8 times its control volume, normalised to unit RMS) and the
radial coordinate r/R to the charge part of the potential (normalised to unit
RMS).  Plain PyTorch CPU operations in float64; no blocking or fusion.

Architecture (levels L, base width C; every 3x3 convolution is bias-free and
followed by ReLU; pooling is the 2x2 average; upsampling repeats each value
2x2; a decoder level concatenates [skip, upsampled] along channels):

    enc_0 = conv(conv(x))                      2 -> C -> C
    enc_l = conv(conv(pool(enc_{l-1})))        C 2^(l-1) -> C 2^l -> C 2^l
    dec_{L-1} = enc_{L-1}
    dec_l = conv(conv(cat(enc_l, up(dec_{l+1}))))   C 2^l + C 2^(l+1) -> C 2^l -> C 2^l
    out = conv1x1(dec_0)                       C -> 1 (no ReLU)

Weights travel as one flat vector, layer by layer in the order above, each
3x3 layer as [c_out][tap][c_in] with tap = 3 (dy + 1) + (dx + 1) the offset of
the input pixel (y + dy, x + dx); the 1x1 layer as [c_in].  Images are
[n][channel][y][x] with y along z (rows) and x along r; they are zero-padded to
multiples of 2^(L-1).
"""
import numpy as np
import torch
import torch.nn.functional as F


def layer_shapes(levels=4, base=16, cin=2):
    """(c_out, c_in, k) of every layer, in the flat-vector order."""
    shapes = []
    c_prev = cin
    for l in range(levels):
        c = base << l
        shapes += [(c, c_prev, 3), (c, c, 3)]
        c_prev = c
    for l in range(levels - 2, -1, -1):
        c = base << l
        shapes += [(c, c + (base << (l + 1)), 3), (c, c, 3)]
    shapes.append((1, base, 1))
    return shapes


def n_params(levels=4, base=16, cin=2):
    return sum(co * ci * k * k for co, ci, k in layer_shapes(levels, base, cin))


def _split(w, levels, base, cin):
    """flat vector -> list of torch conv weights [c_out][c_in][kh][kw]"""
    out, o = [], 0
    for co, ci, k in layer_shapes(levels, base, cin):
        n = co * ci * k * k
        a = torch.as_tensor(np.asarray(w[o:o + n], dtype=np.float64)).reshape(co, k * k, ci)
        out.append(a.permute(0, 2, 1).reshape(co, ci, k, k))  # tap = 3 ky + kx
        o += n
    assert o == len(w)
    return out


def _join(grads):
    parts = []
    for g in grads:
        co, ci, k, _ = g.shape
        parts.append(g.reshape(co, ci, k * k).permute(0, 2, 1).reshape(-1))
    return torch.cat(parts).numpy()


def _conv(x, w):
    # cross-correlation: out[y, x] = sum over taps of w[dy+1, dx+1] in[y+dy, x+dx]
    return F.conv2d(x, w, padding=w.shape[-1] // 2)


def bf16_round(t):
    """round a float64 tensor to the nearest-even BF16 value (through FP32)"""
    a = t.detach().to(torch.float32).contiguous().view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    a = ((a + 0x7FFF + ((a >> 16) & 1)) >> 16) << 16
    a = torch.where(a >= 2 ** 31, a - 2 ** 32, a).to(torch.int32)
    return a.view(torch.float32).to(torch.float64)


def _store(h, rounding):
    # activations kept in a storage precision: rounded forward, gradient
    # passed straight through
    if rounding is None:
        return h
    return h + (bf16_round(h) - h).detach()


def forward_t(x, ws, levels, rounding=None):
    enc, h, k = [], _store(x, rounding), 0
    for l in range(levels):
        if l > 0:
            h = _store(F.avg_pool2d(h, 2), rounding)
        h = _store(F.relu(_conv(h, ws[k])), rounding)
        h = _store(F.relu(_conv(h, ws[k + 1])), rounding)
        k += 2
        enc.append(h)
    d = enc[-1]
    for l in range(levels - 2, -1, -1):
        u = F.interpolate(d, scale_factor=2, mode="nearest")
        h = torch.cat([enc[l], u], dim=1)
        h = _store(F.relu(_conv(h, ws[k])), rounding)
        d = _store(F.relu(_conv(h, ws[k + 1])), rounding)
        k += 2
    return _conv(d, ws[k])


def forward(x, w, levels=4, base=16, rounding=None):
    """x: [n][cin][H][W] float64 numpy -> [n][1][H][W]; rounding="bf16" keeps
    the input and every activation in BF16 (the storage precision of a BF16
    implementation), all arithmetic in float64"""
    xt = torch.as_tensor(np.asarray(x, dtype=np.float64))
    ws = _split(w, levels, base, xt.shape[1])
    with torch.no_grad():
        return forward_t(xt, ws, levels, rounding).numpy()


def weight_gradient(x, w, dout, levels=4, base=16, rounding=None):
    """d(sum(dout * out)) / dw, flat, in the weight order; and d/dx."""
    xt = torch.as_tensor(np.asarray(x, dtype=np.float64)).clone().requires_grad_(True)
    ws = [t.clone().requires_grad_(True) for t in _split(w, levels, base, xt.shape[1])]
    out = forward_t(xt, ws, levels, rounding)
    (out * torch.as_tensor(np.asarray(dout, dtype=np.float64))).sum().backward()
    return _join([t.grad for t in ws]), xt.grad.numpy()


def padded_size(nr, nz, levels=4):
    """image size (H = z nodes, W = r nodes) padded to multiples of 2^(L-1)"""
    m = 1 << (levels - 1)
    H = -(-(nz + 1) // m) * m
    W = -(-(nr + 1) // m) * m
    return H, W


def sample(o, Q, phi_p, levels=4):
    """Network input and target for node charge Q and the charge part of the
    potential phi_p (both [(nz+1)][(nr+1)]) of oracle o:
      channel 0: b = w_i rho / eps0 on the interior rows (w_i = A_i dz the
                 node's control volume, rho = Q qunit / V_node), over its RMS;
      channel 1: r / R on the real nodes;
      target:    phi_p on the interior rows over its RMS.
    Everything outside the real nodes is zero.  Returns (x [2][H][W], y [H][W])."""
    nr, nz = o.nr, o.nz
    H, W = padded_size(nr, nz, levels)
    dr, dz = o.R / nr, o.L / nz
    Vn, _ = o.node_volumes()
    lo = np.maximum(np.arange(nr + 1) - 0.5, 0.0) * dr
    hi = np.minimum(np.arange(nr + 1) + 0.5, nr) * dr
    w = (hi * hi - lo * lo) / 2.0 * dz
    qunit = 1.602176634e-19 * o.weight * 2.0 ** -40
    b = np.zeros((nz + 1, nr + 1))
    b[1:nz] = w[None, :] * ((np.asarray(Q, np.float64)[1:nz] * qunit / Vn[None, :]) / 8.8541878128e-12)
    x = np.zeros((2, H, W))
    rb = np.sqrt(np.mean(b[1:nz] ** 2))
    x[0, :nz + 1, :nr + 1] = b / rb if rb > 0 else b
    x[1, :nz + 1, :nr + 1] = (np.arange(nr + 1) / nr)[None, :]
    y = np.zeros((H, W))
    t = np.asarray(phi_p, np.float64)
    rt = np.sqrt(np.mean(t[1:nz] ** 2))
    y[1:nz, :nr + 1] = t[1:nz] / rt if rt > 0 else t[1:nz]
    return x, y
