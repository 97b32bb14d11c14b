"""Learned fine-level smoother (not in the paper): the plain definition the GPU
library is checked against.  TEST INFRASTRUCTURE ONLY (see the package header).

Per face F of the finest level a two-layer network maps a window of the current
residual r to a correction of F's velocity unknowns:

* window of F: for each side s = 0, 1 (the cells T_0, T_1 of F in increasing
  cell order; T_1 absent on the boundary) the residual blocks of the faces of
  T_s in the cell's face order, padded with zeros to ``Fm`` = max faces per
  cell, then the residual of T_s's pressure unknowns; after both sides, a
  one-hot of F's position in T_0's face list and in T_1's.  With d components,
  p face modes and t pressure modes per cell the window has
  n_in = 2 (Fm d p + t) + 2 Fm entries (370 + 12 = 412 for 3D hexahedra, k = 3,
  v-cond);
* scale: s_F = sqrt(mean of the squared residual entries of the window, the
  zero padding included, i.e. over 2 (Fm d p + t) entries); the residual part
  is divided by s_F, the one-hot part is not;
* network: h = relu(W1 x + b1) (64 hidden units), y = W2 h + b2 with
  d p + 2 t outputs: the correction of F's velocity unknowns, then of the
  pressure unknowns of T_0 and of T_1 (the pressure head);
* correction: delta_F = s_F y[:d p] (0 when s_F = 0); every cell T takes the
  mean over its faces F of s_F y_F[d p + side t : d p + (side + 1) t], side the
  position of T in F's cell pair.
* precision: the network runs on bfloat16 weights and activations with sums
  kept exact here (FP32 on the GPU): x, W1, W2 and h are rounded to bfloat16
  (``round_bf16`` of oracle.mixed, from float32), biases and outputs are not;
  the gradients are those of this network with each rounding taken as the
  identity.  ``quantize=False`` gives the unrounded FP64 network.

Training data are pairs (window of r, e_F / s_F) with e the error of the
current iterate (its velocity block on F, then its pressure blocks on T_0 and
T_1, 0 for an absent T_1); the loss is 1/(2B) sum_i |y_i - t_i|^2 over a batch of
B samples; parameters are updated with Adam (Kingma & Ba 2015: beta1 = 0.9,
beta2 = 0.999, eps = 1e-8, bias-corrected moments) on FP32 master values.

Inside the V-cycle the correction is one more search direction of the
fine-level smoothing step: the step minimises the residual over
span{M r, M A M r, N(r)} (M the Schwarz preconditioner), so it can never do
worse than the plain step over span{M r, M A M r}.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

HIDDEN = 64


@dataclass
class Layout:
    d: int
    p: int
    t: int
    Fm: int
    nface: int     # offset of the cell pressure part in a level vector

    @property
    def dp(self):
        return self.d * self.p

    @property
    def n_res(self):
        return 2 * (self.Fm * self.dp + self.t)

    @property
    def n_in(self):
        return self.n_res + 2 * self.Fm

    @property
    def n_out(self):
        return self.dp + 2 * self.t


def layout(mesh, d: int, p: int, t: int) -> Layout:
    Fm = int(np.diff(mesh.cell_ptr).max())
    return Layout(d, p, t, Fm, mesh.n_faces * d * p)


def windows(mesh, L: Layout, r: np.ndarray):
    """X [nf, n_in] (residual part scaled by s), s [nf]."""
    fc = mesh.face_cells()
    nf = mesh.n_faces
    X = np.zeros((nf, L.n_in))
    s = np.zeros(nf)
    side = L.Fm * L.dp + L.t
    for f in range(nf):
        for si in range(2):
            c = fc[f, si]
            if c < 0:
                continue
            faces = list(mesh.cell_faces(c))
            o = si * side
            for i, g in enumerate(faces):
                X[f, o + i * L.dp:o + (i + 1) * L.dp] = r[g * L.dp:(g + 1) * L.dp]
            X[f, o + L.Fm * L.dp:o + side] = r[L.nface + c * L.t:L.nface + (c + 1) * L.t]
            X[f, L.n_res + si * L.Fm + faces.index(f)] = 1.0
        s[f] = np.sqrt(np.sum(X[f, :L.n_res] ** 2) / L.n_res)
        if s[f] > 0:
            X[f, :L.n_res] /= s[f]
    return X, s


def init_params(n_in: int, n_out: int, u1: np.ndarray, u2: np.ndarray):
    """He-uniform weights from given uniform(0,1) draws (u1 [H*n_in], u2 [n_out*H]); zero biases."""
    a1 = np.sqrt(6.0 / n_in)
    a2 = np.sqrt(6.0 / HIDDEN)
    W1 = (2.0 * u1.reshape(HIDDEN, n_in) - 1.0) * a1
    W2 = (2.0 * u2.reshape(n_out, HIDDEN) - 1.0) * a2
    return dict(W1=W1, b1=np.zeros(HIDDEN), W2=W2, b2=np.zeros(n_out))


def _bf(a):
    from .mixed import round_bf16
    return round_bf16(np.asarray(a, dtype=np.float32)).astype(np.float64)


def forward(th, X, quantize=True):
    """Y, Z (pre-activations), H (activations as the second layer reads them)."""
    q = _bf if quantize else (lambda a: a)
    Z = q(X) @ q(th["W1"]).T + th["b1"]
    H = q(np.maximum(Z, 0.0))
    return H @ q(th["W2"]).T + th["b2"], Z, H


def loss_and_grad(th, X, T, quantize=True):
    """Loss 1/(2B) sum |Y - T|^2 and its gradient (backpropagation written out;
    the bfloat16 roundings are taken as the identity)."""
    q = _bf if quantize else (lambda a: a)
    B = X.shape[0]
    Y, Z, H = forward(th, X, quantize)
    D = Y - T
    loss = 0.5 * np.sum(D * D) / B
    dY = D / B
    gW2 = dY.T @ H
    gb2 = dY.sum(axis=0)
    dZ = (dY @ q(th["W2"])) * (Z > 0)
    gW1 = dZ.T @ q(X)
    gb1 = dZ.sum(axis=0)
    return loss, dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2)


def adam_step(th, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (th, m, v)."""
    th2, m2, v2 = {}, {}, {}
    for k in th:
        m2[k] = b1 * m[k] + (1 - b1) * g[k]
        v2[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m2[k] / (1 - b1 ** step)
        vh = v2[k] / (1 - b2 ** step)
        th2[k] = th[k] - lr * mh / (np.sqrt(vh) + eps)
    return th2, m2, v2


def apply(th, mesh, L: Layout, r: np.ndarray, quantize=True) -> np.ndarray:
    """Level-0 vector: delta_F on every face block, the mean of the pressure
    outputs of a cell's faces on its pressure block."""
    X, s = windows(mesh, L, r)
    Y, _, _ = forward(th, X, quantize)
    z = np.zeros_like(r)
    z[:L.nface] = (s[:, None] * Y[:, :L.dp]).ravel()
    fc = mesh.face_cells()
    for c in range(mesh.n_cells):
        faces = list(mesh.cell_faces(c))
        acc = np.zeros(L.t)
        for f in faces:
            side = 0 if fc[f, 0] == c else 1
            acc += s[f] * Y[f, L.dp + side * L.t:L.dp + (side + 1) * L.t]
        z[L.nface + c * L.t:L.nface + (c + 1) * L.t] = acc / len(faces)
    return z


def targets(mesh, L: Layout, e: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Training targets of every face: (e_F, e_T0, e_T1) / s_F (0 where s_F = 0
    and for an absent T_1)."""
    fc = mesh.face_cells()
    T = np.zeros((mesh.n_faces, L.n_out))
    for f in range(mesh.n_faces):
        if s[f] <= 0:
            continue
        T[f, :L.dp] = e[f * L.dp:(f + 1) * L.dp] / s[f]
        for side in range(2):
            c = fc[f, side]
            if c >= 0:
                T[f, L.dp + side * L.t:L.dp + (side + 1) * L.t] = e[L.nface + c * L.t:L.nface + (c + 1) * L.t] / s[f]
    return T


def mr_step(A, dirs, x, r):
    """x + Z y with y minimising |r - A Z y| over the given directions (least squares)."""
    W = np.stack([A(z) for z in dirs], axis=1)
    y, *_ = np.linalg.lstsq(W, r, rcond=None)
    return x + np.stack(dirs, axis=1) @ y
