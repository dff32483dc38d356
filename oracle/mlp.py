"""FP64 reference of the learned warm start: a 7-128-128-3 tanh network, its
loss gradient, the Adam update, bfloat16 inference and the warm-start fields
(density and velocity) built from it.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component; this network is an extension that
proposes the initial density of a static drop (Sec. 5.3) so that the solver
reaches its converged state in fewer steps.  What it computes follows
published definitions:

* the network: z1 = W1 x + b1, a1 = tanh z1, z2 = W2 a1 + b2, a2 = tanh z2,
  y = W3 a2 + b3 (three outputs), loss = mean over samples of
  sum_j (y_j - t_j)^2;
* gradients by the chain rule (backpropagation), written out layer by layer;
* Adam (Kingma and Ba, ICLR 2015, Algorithm 1) with bias correction;
* bfloat16 = the upper 16 bits of an IEEE binary32 after rounding to
  nearest, ties to even.

Flat parameter vector (float32 on the device, float64 here), in this order:
W1 (128 x 7, row = output unit), b1 (128), W2 (128 x 128), b2 (128),
W3 (3 x 128), b3 (3): 17 923 values.

Features of a node of a drop: (T/Tc, R / 256, kappa, k, r - R, cos 4 theta,
sin 4 theta), theta the polar angle about the drop's centre.  Outputs: the
normalised log density (ln rho - ln rho_g) / (ln rho_l - ln rho_g) and the
radial and azimuthal fluid velocity v = u + F/(2 rho) in units of 1e-3.  The angle enters through
4 theta because a drop centred in a square periodic mesh keeps the square's
symmetry, and so does its steady velocity field.
"""
import numpy as np

N_IN, N_HID, N_OUT = 7, 128, 3
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)

# feature normalisation: x_i = (f_i - CENTER_i) / SCALE_i
FEATURE_CENTER = np.array([0.5, 0.25, 0.1, 0.25, 0.0, 0.0, 0.0])
FEATURE_SCALE = np.array([0.25, 0.1, 0.1, 0.1, 8.0, 1.0, 1.0])
R_REF = 256.0
U_SCALE = 1e-3


def unpack(w):
    """Views of the flat vector as (W1, b1, W2, b2, W3, b3)."""
    out, o = [], 0
    for _, s in SHAPES:
        n = int(np.prod(s))
        out.append(w[o:o + n].reshape(s))
        o += n
    return out


def forward(w, x):
    """y (n, 3) and the activations (a1, a2) for samples x (n, 7)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(w, dtype=np.float64))
    a1 = np.tanh(x @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    return a2 @ W3.T + b3, a1, a2


def loss(w, x, t):
    y, _, _ = forward(w, x)
    return float(np.sum((y - t) ** 2) / x.shape[0])


def grad(w, x, t):
    """(loss, dloss/dw as a flat vector) by backpropagation."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(w, dtype=np.float64))
    y, a1, a2 = forward(w, x)
    n = x.shape[0]
    dy = 2.0 * (y - t) / n                # dL/dy, (n, 3)
    gW3 = dy.T @ a2                       # dL/dW3[j, u] = sum_s dy[s, j] a2[s, u]
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * (1.0 - a2 * a2)     # through y = W3 a2 and tanh
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - a1 * a1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(np.sum((y - t) ** 2) / n), g


def adam(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16(a):
    """Round binary32 values to bfloat16 (nearest, ties to even); returned as
    float64 holding the rounded value.  The input is first rounded to
    binary32, as the device holds it."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(w, x):
    """Inference with the hidden-to-hidden product in bfloat16: W2 and a1 are
    rounded to bfloat16, their products summed exactly (here in FP64); the
    other layers as in forward()."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(w, dtype=np.float32).astype(np.float64))
    a1 = np.tanh(np.asarray(x, dtype=np.float32).astype(np.float64) @ W1.T + b1)
    a2 = np.tanh(bf16(a1) @ bf16(W2).T + b2)
    return a2 @ W3.T + b3


def drop_geometry(radius, nx, ny, cx=None, cy=None):
    """(r - R, theta) of every node (ny*nx,) of a drop of `radius` centred
    at (cx, cy) (default the domain centre); plain distances."""
    cx = nx / 2.0 if cx is None else cx
    cy = ny / 2.0 if cy is None else cy
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    dx, dy = (x - cx).ravel(), (y - cy).ravel()
    return np.sqrt(dx * dx + dy * dy) - radius, np.arctan2(dy, dx)


def drop_features(T_r, radius, kappa, k, nx, ny, cx=None, cy=None):
    """Normalised features (ny*nx, 7) of every node of a drop."""
    d, th = drop_geometry(radius, nx, ny, cx, cy)
    f = np.empty((nx * ny, N_IN))
    f[:, 0] = T_r
    f[:, 1] = radius / R_REF
    f[:, 2] = kappa
    f[:, 3] = k
    f[:, 4] = d
    f[:, 5] = np.cos(4.0 * th)
    f[:, 6] = np.sin(4.0 * th)
    return (f - FEATURE_CENTER) / FEATURE_SCALE


def symmetric_outputs(w, x, bf16=True):
    """Outputs made symmetric under the square's reflections about the drop's
    centre, which map (cos 4 theta, sin 4 theta) to (cos 4 theta,
    -sin 4 theta): with y+ at x and y- at x with its last feature negated,
    (y0, y1) are the even parts and y2 the odd part."""
    xm = np.array(x, dtype=np.float64)
    xm[:, -1] = -xm[:, -1]
    fwd = forward_bf16 if bf16 else (lambda w_, x_: forward(w_, x_)[0])
    yp, ym = fwd(w, x), fwd(w, xm)
    y = 0.5 * (yp + ym)
    y[:, 2] = 0.5 * (yp[:, 2] - ym[:, 2])
    return y


def velocity_from_output(y, theta):
    """(ux, uy) from the radial and azimuthal outputs (units of U_SCALE)."""
    ur, ut = U_SCALE * y[:, 1], U_SCALE * y[:, 2]
    c, s = np.cos(theta), np.sin(theta)
    return ur * c - ut * s, ur * s + ut * c


def drop_velocity(y, radius, nx, ny, cx=None, cy=None):
    """Velocity field (ny, nx) x 2 of a drop from symmetric outputs: the polar
    components rotated to (ux, uy), with the x (y) velocity zero on nodes
    that are their own mirror image about x = cx (y = cy) in the periodic
    mesh -- the centre column (row) and, for cx = nx/2 (cy = ny/2), the edge
    column (row) -- as mirror symmetry demands."""
    cx = nx / 2.0 if cx is None else cx
    cy = ny / 2.0 if cy is None else cy
    _, th = drop_geometry(radius, nx, ny, cx, cy)
    ux, uy = velocity_from_output(y, th)
    ux, uy = ux.reshape(ny, nx), uy.reshape(ny, nx)
    xs, ys = np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64)
    ux[:, np.fmod(2.0 * (xs - cx), nx) == 0.0] = 0.0
    uy[np.fmod(2.0 * (ys - cy), ny) == 0.0, :] = 0.0
    return ux, uy


REACH_BLEND = 10.0


def reach_weight(radius, nx, ny, reach, cx=None, cy=None):
    """Weight (ny*nx,) of the network's outputs for a network used within
    `reach` nodes of the interface: 1 where r - R <= reach - REACH_BLEND, 0
    where r - R >= reach + REACH_BLEND, linear in r between; 1 everywhere
    for an infinite reach.  Scaling the outputs by it leaves the Maxwell gas
    at rest beyond the blend."""
    d, _ = drop_geometry(radius, nx, ny, cx, cy)
    if np.isinf(reach):
        return np.ones_like(d)
    return np.clip((reach + REACH_BLEND - d) / (2.0 * REACH_BLEND), 0.0, 1.0)


def density_from_output(y, rho_g, rho_l):
    """The network predicts the normalised log density
    y = (ln rho - ln rho_g) / (ln rho_l - ln rho_g)."""
    return np.exp(np.log(rho_g) + y * (np.log(rho_l) - np.log(rho_g)))


def mass_match(rho, target_mass, rho_g, rho_l):
    """Add target - sum(rho) in proportion to w = max((rho - rho_g)(rho_l - rho), 0),
    a weight that vanishes in both bulks (the interface absorbs the
    difference)."""
    wgt = np.maximum((rho - rho_g) * (rho_l - rho), 0.0)
    return rho + (target_mass - rho.sum()) * wgt / wgt.sum()
