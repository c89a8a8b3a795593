"""The learned proposal's network, forward and analytic backward in FP64
(test infrastructure; NumPy).

Network 1 -> 64 -> 64 -> 33 on t = alpha / ALPHA_MAX:
    h1 = silu(W1 t + b1), h2 = silu(W2 h1 + b2), z = W3 h2 + b3,
    silu(a) = a / (1 + exp(-a)).
The first 32 outputs give the widths of the proposal's 32 equal-probability
segments of x0 on [-1, 1]: w = 2 softmax(z[0:32]), knots
y_0 = -1, y_j = -1 + sum_{i<j} w_i (so y_32 = +1).  Output 32 is reserved: it
enters neither the proposal nor the loss.
Loss: L = mean over samples and the 32 segments of (log w_j - log w*_j)^2,
with w* the widths of the integrated CDF's knots (oracle/cdf.py).

Parameters travel as one flat vector in the order W1 (64x1), b1 (64),
W2 (64x64), b2 (64), W3 (33x64), b3 (33): 6433 numbers, row-major.  The GPU
evaluates the network with the weights rounded to BF16; the oracle takes the
same rounded values (bf16_round) so the two compute the same function.
"""
import numpy as np

ALPHA_MAX = 40.0
H = 64
NOUT = 33
NSEG = 32
SHAPES = [("W1", (H, 1)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (NOUT, H)),
          ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)  # 6433


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAM,)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(params[n], dtype=np.float64).ravel() for n, _ in SHAPES])


def bf16_round(x):
    """Round float32 values to the nearest BF16 (ties to even), returned as
    float64.  BF16 keeps the top 16 bits of the float32 pattern."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def forward(theta, alphas):
    """Returns (knots [n, 33], log widths [n, 32], cache)."""
    p = unpack(theta)
    t = np.asarray(alphas, dtype=np.float64)[:, None] / ALPHA_MAX
    a1 = t @ p["W1"].T + p["b1"]
    h1 = a1 * _sigmoid(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = a2 * _sigmoid(a2)
    z = h2 @ p["W3"].T + p["b3"]
    zs = z[:, :NSEG]
    m = zs.max(axis=1, keepdims=True)
    lse = m + np.log(np.sum(np.exp(zs - m), axis=1, keepdims=True))
    logw = np.log(2.0) + zs - lse
    w = np.exp(logw)
    y = np.concatenate([-np.ones((len(t), 1)), -1.0 + np.cumsum(w, axis=1)], axis=1)
    y[:, -1] = 1.0
    cache = dict(t=t, a1=a1, h1=h1, a2=a2, h2=h2, z=z, logw=logw, p=p)
    return y, logw, cache


def loss_and_grad(theta, alphas, target_logw):
    """L and dL/dtheta (flat, same order as theta)."""
    y, logw, c = forward(theta, alphas)
    p = c["p"]
    n = len(c["t"])
    e = logw - np.asarray(target_logw, dtype=np.float64)
    L = float(np.mean(e * e))
    # dL/dlogw_j = 2 e_j / (n NSEG); logw_j = log 2 + z_j - lse -> dL/dz_i = g_i - softmax_i sum_j g_j
    g = 2.0 * e / (n * NSEG)
    sm = np.exp(logw) / 2.0
    dz = np.zeros_like(c["z"])
    dz[:, :NSEG] = g - sm * g.sum(axis=1, keepdims=True)
    dW3 = dz.T @ c["h2"]
    db3 = dz.sum(axis=0)
    dh2 = dz @ p["W3"]
    s2 = _sigmoid(c["a2"])
    da2 = dh2 * (s2 * (1.0 + c["a2"] * (1.0 - s2)))
    dW2 = da2.T @ c["h1"]
    db2 = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    s1 = _sigmoid(c["a1"])
    da1 = dh1 * (s1 * (1.0 + c["a1"] * (1.0 - s1)))
    dW1 = da1.T @ c["t"]
    db1 = da1.sum(axis=0)
    grad = pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))
    return L, grad


# ---------------------------------------------------------------------------
# Training: full-batch Adam (Kingma & Ba, "Adam: a method for stochastic
# optimization", ICLR 2015, Algorithm 1) with a cosine learning-rate decay.
# The master parameters are held in FP64; every step evaluates the loss and
# gradient at their BF16 rounding, the values the network computes with.
# ---------------------------------------------------------------------------
ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8


def cosine_lr(t, total, lr0, lr_min):
    """Learning rate of step t = 1, 2, ...: lr0 at t = 1, falling along half
    a cosine period to lr_min at t = total + 1 (and held there after)."""
    frac = min(1.0, (t - 1) / max(1, total))
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + np.cos(np.pi * frac))


def adam_step(theta, g, m, v, t, lr):
    """Step t >= 1 of Adam: moment estimates m, v updated with gradient g,
    bias-corrected by 1 - beta^t, then theta moves by lr m_hat / (sqrt(v_hat)
    + eps).  Returns the new (theta, m, v)."""
    g = np.asarray(g, dtype=np.float64)
    m = ADAM_BETA1 * m + (1.0 - ADAM_BETA1) * g
    v = ADAM_BETA2 * v + (1.0 - ADAM_BETA2) * g * g
    m_hat = m / (1.0 - ADAM_BETA1 ** t)
    v_hat = v / (1.0 - ADAM_BETA2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + ADAM_EPS), m, v


def train(theta0, alphas, target_logw, steps, lr0, lr_min):
    """`steps` Adam steps from theta0 with zero initial moments, the
    gradient of each taken at the BF16 rounding of the current parameters.
    Returns (final FP64 master parameters, loss before each step)."""
    theta = np.asarray(theta0, dtype=np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for t in range(1, steps + 1):
        L, g = loss_and_grad(bf16_round(theta), alphas, target_logw)
        hist.append(L)
        theta, m, v = adam_step(theta, g, m, v, t, cosine_lr(t, steps, lr0, lr_min))
    return theta, np.array(hist)
