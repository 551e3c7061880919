"""FP64 reference of the order/leaf-capacity predictor -- TEST INFRASTRUCTURE.

A plain NumPy FP64 implementation of the network the learned mode uses:
input standardisation, two hidden ReLU layers and two softmax heads (order
class and leaf-capacity class), the mean of the two cross-entropy losses,
its analytic gradient, and one Adam update (Kingma & Ba, 2015: biased first
and second moments, bias correction, eps added to the corrected root).

Parameter vector layout (shared with the device kernels by definition of the
interface, not by code): mean[F], std[F], W1[F][H], b1[H], W2[H][H], b2[H],
W3[H][C], b3[C] with F = 12 inputs, H = 64, C = 8 logits (4 + 4).
"""
import numpy as np

F, H, C = 12, 64, 8
HEADS = ((0, 4), (4, 8))


def sizes():
    return [("mean", (F,)), ("std", (F,)), ("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
            ("W3", (H, C)), ("b3", (C,))]


def nparam():
    return sum(int(np.prod(s)) for _, s in sizes())


def unpack(theta):
    out, k = {}, 0
    for name, s in sizes():
        n = int(np.prod(s))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(s)
        k += n
    return out


def forward(theta, X):
    P = unpack(theta)
    Z = (np.asarray(X, dtype=np.float64) - P["mean"]) / P["std"]
    A1 = Z @ P["W1"] + P["b1"]
    H1 = np.maximum(A1, 0.0)
    A2 = H1 @ P["W2"] + P["b2"]
    H2 = np.maximum(A2, 0.0)
    logits = H2 @ P["W3"] + P["b3"]
    return logits, (Z, A1, H1, A2, H2)


def loss_and_grad(theta, X, labels):
    """Mean over rows of (CE(order head) + CE(capacity head)) / 2 and its
    gradient with respect to the trainable parameters (mean/std get 0)."""
    P = unpack(theta)
    logits, (Z, A1, H1, A2, H2) = forward(theta, X)
    B = len(Z)
    dlog = np.zeros_like(logits)
    loss = 0.0
    for h, (a, b) in enumerate(HEADS):
        l = logits[:, a:b]
        m = l.max(axis=1, keepdims=True)
        e = np.exp(l - m)
        s = e / e.sum(axis=1, keepdims=True)
        y = np.asarray(labels)[:, h]
        loss += -np.mean(np.log(s[np.arange(B), y]))
        g = s.copy()
        g[np.arange(B), y] -= 1.0
        dlog[:, a:b] = g / B
    loss *= 0.5
    dlog *= 0.5
    grads = {"mean": np.zeros(F), "std": np.zeros(F)}
    grads["W3"] = H2.T @ dlog
    grads["b3"] = dlog.sum(axis=0)
    dH2 = (dlog @ P["W3"].T) * (A2 > 0)
    grads["W2"] = H1.T @ dH2
    grads["b2"] = dH2.sum(axis=0)
    dH1 = (dH2 @ P["W2"].T) * (A1 > 0)
    grads["W1"] = Z.T @ dH1
    grads["b1"] = dH1.sum(axis=0)
    g = np.concatenate([grads[name].reshape(-1) for name, _ in sizes()])
    return loss, g


def adam(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); mean/std are not trained."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    with np.errstate(divide="ignore", invalid="ignore"):
        upd = lr * mhat / (np.sqrt(vhat) + eps)
    upd[: 2 * F] = 0.0
    upd[np.isnan(upd)] = 0.0
    return theta - upd, m, v


def init(seed, mean=None, std=None):
    """He-initialised parameters with the given input standardisation."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, s in sizes():
        if name == "mean":
            parts.append(np.zeros(F) if mean is None else np.asarray(mean, float))
        elif name == "std":
            parts.append(np.ones(F) if std is None else np.asarray(std, float))
        elif name.startswith("W"):
            parts.append(rng.standard_normal(s).reshape(-1) * np.sqrt(2.0 / s[0]))
        else:
            parts.append(np.zeros(int(np.prod(s))))
    return np.concatenate(parts)
