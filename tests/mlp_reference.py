"""FP64 CPU reference of the prescreener network (test infrastructure).

Same architecture and parameter layout as the library: 12 -> 64 -> 64 -> 64 -> 1,
SiLU hidden activations, pinball loss at quantile q on (target - prediction).
With `rounding=True` the weights, the standardised inputs and the hidden
activations are rounded to bf16 as in the library's kernels (gradients pass
straight through the rounding)."""
import numpy as np

NF, NH = 12, 64
SIZES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NH)), ("b3", (NH,)),
         ("w4", (NH,)), ("b4", (1,))]


def unpack(p):
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def bf16(x):
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1 + np.exp(-z))


def dsilu(z):
    s = 1 / (1 + np.exp(-z))
    return s * (1 + z * (1 - s))


def loss_and_grad(p, X, y, mean, std, q, rounding=True):
    P = unpack(p)
    r = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    W1, W2, W3, w4 = r(P["W1"]), r(P["W2"]), r(P["W3"]), r(P["w4"])
    x = r((np.asarray(X, np.float32) - np.asarray(mean, np.float32)) * (np.float32(1) / np.asarray(std, np.float32)))
    z1 = x @ W1.T + P["b1"]
    a1 = r(silu(z1))
    z2 = a1 @ W2.T + P["b2"]
    a2 = r(silu(z2))
    z3 = a2 @ W3.T + P["b3"]
    a3 = r(silu(z3))
    yp = a3 @ w4 + P["b4"][0]
    res = y - yp
    B = len(y)
    loss = np.where(res > 0, q * res, (q - 1) * res)
    gy = np.where(res > 0, -q, 1 - q) / B
    d3 = gy[:, None] * w4[None, :] * dsilu(z3)
    d2 = (d3 @ W3) * dsilu(z2)
    d1 = (d2 @ W2) * dsilu(z1)
    g = {"W1": d1.T @ x, "b1": d1.sum(0), "W2": d2.T @ a1, "b2": d2.sum(0), "W3": d3.T @ a2, "b3": d3.sum(0),
         "w4": gy @ a3, "b4": np.array([gy.sum()])}
    flat = np.concatenate([g[name].ravel() for name, _ in SIZES])
    return loss.mean(), flat, yp
