"""Plain FP64 reference of the learned-closure pieces (test infrastructure:
only the tests, the smoke check and the benchmark's CPU baseline use it).

The learned closure is an extension beyond the paper (which resolves every
fiber, Sec. 4.2); what is defined here is the network of that extension and
its input features, written out directly with numpy:

  * network 247 -> 64 -> 64 -> 6 with the exact GELU g(z) = z Phi(z) after
    the hidden layers, parameters packed as W1[64][247], b1, W2[64][64], b2,
    W3[6][64], b3;
  * inputs normalised as (x - mean) * inv_std, outputs multiplied by
    out_scale;
  * mean squared error and its gradient by the chain rule (pinned in the
    tests by central finite differences);
  * Adam (Kingma and Ba 2015) in FP32 arithmetic;
  * BF16 round-to-nearest-even of FP32 values;
  * the features of a fiber from a velocity field: velocities relative to
    the rigid motion on the 3 x 27 stencil (centre and tips, offsets
    {-2, 0, 2}^3 along the body axes, trilinear, z clamped), in the body
    frame, divided by gamma L, and the quaternion with w >= 0.
"""
import numpy as np
from scipy.special import erf

NI, NH, NO = 247, 64, 6
NPARAM = NH * NI + NH + NH * NH + NH + NO * NH + NO


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + NH * NI].reshape(NH, NI); o += NH * NI
    b1 = w[o:o + NH]; o += NH
    W2 = w[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = w[o:o + NH]; o += NH
    W3 = w[o:o + NO * NH].reshape(NO, NH); o += NO * NH
    b3 = w[o:o + NO]; o += NO
    assert o == NPARAM
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def bf16_round(x):
    """FP32 values rounded to BF16 (nearest, ties to even), back as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward(w, xn):
    """Network outputs (raw, before out_scale) for normalised inputs xn[n][247]."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    z1 = xn @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    return h2 @ W3.T + b3


def loss_grad(w, xn, t):
    """Mean squared error over n x 6 outputs against t, and its gradient."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    n = xn.shape[0]
    z1 = xn @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    y = h2 @ W3.T + b3
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / (n * NO)
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dz2 = (dy @ W3) * gelu_d(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * gelu_d(z1)
    gW1 = dz1.T @ xn
    gb1 = dz1.sum(0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in FP32 (step number t >= 1); returns new w, m, v."""
    f = np.float32
    w, m, v, g = (np.asarray(a, dtype=f) for a in (w, m, v, g))
    m = f(b1) * m + f(1 - b1) * g
    v = f(b2) * v + f(1 - b2) * g * g
    c1, c2 = f(1 - b1 ** t), f(1 - b2 ** t)
    w = w - f(lr) * (m / c1) / (np.sqrt(v / c2) + f(eps))
    return w, m, v


def rotation(q):
    """R(q) for a unit quaternion (w, x, y, z): columns are the body axes."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def features(u, X, q, V, W, length, gamma):
    """Features [247] of one fiber from the velocity field u[3][nz][ny][nx]
    (fiber cells holding the rigid-body velocity), periodic in x, y:
    relative velocities at X + s t + R(q) o (s in 0, L/2, -L/2; o in
    {-2,0,2}^3), in the body frame, over gamma L; then q with w >= 0."""
    _, nz, ny, nx = u.shape
    R = rotation(np.asarray(q, dtype=np.float64))
    out = np.zeros(247)
    L = float(length)
    for pt, side in enumerate((0.0, 0.5 * L, -0.5 * L)):
        for m in range(27):
            ob = 2.0 * np.array([m % 3 - 1, (m // 3) % 3 - 1, m // 9 - 1])
            d = side * R[:, 0] + R @ ob
            p = np.asarray(X, dtype=np.float64) + d
            pz = min(max(p[2], 0.0), nz - 1.0)
            x0, y0 = int(np.floor(p[0])), int(np.floor(p[1]))
            z0 = min(int(np.floor(pz)), nz - 2)
            ax, ay, az = p[0] - x0, p[1] - y0, pz - z0
            val = np.zeros(3)
            for c in range(8):
                cx, cy, cz = c & 1, (c >> 1) & 1, c >> 2
                wgt = (ax if cx else 1 - ax) * (ay if cy else 1 - ay) * (az if cz else 1 - az)
                val += wgt * u[:, z0 + cz, (y0 + cy) % ny, (x0 + cx) % nx]
            us = np.asarray(V) + np.cross(W, d)
            k = pt * 27 + m
            out[3 * k:3 * k + 3] = R.T @ (val - us) / (gamma * L)
    qq = np.asarray(q, dtype=np.float64)
    out[243:] = -qq if qq[0] < 0 else qq
    return out
