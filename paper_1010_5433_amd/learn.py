"""Training and evaluation of the learned preconditioner.

Everything numerical runs in the library's kernels: the training pairs are
made with the library's double precision operator and solver, the network
is trained by its forward, backward and Adam kernels, and it is evaluated inside
its flexible CG.  This module only drives those calls.

Training pairs.  For a source/solution pair (b, x) of M x = b the loss
||P(b) - x||^2 / ||x||^2 weighs each eigenmode of M by the size of its
component in x.  With x drawn white and b = M x the loss is the mean of
|1 - lambda p(lambda)|^2 over the spectrum, which is what a preconditioner of
CG needs; with b drawn white (x = M^-1 b from the solver) the low modes carry
weights 1/lambda^2, and the fitted network is in general not positive
definite.  make_pairs therefore draws x and forms b = M x in double
precision; solve_pairs (b white, x from the solver) is kept for comparison.
"""
from __future__ import annotations

import time

import torch

from . import Lattice, Net, NET_NPARAM


def _white(shape, gen, device="cuda"):
    """Complex Gaussian library vectors (float64), unit variance per complex entry."""
    return torch.randn(shape, generator=gen, dtype=torch.float64, device=device) * (0.5 ** 0.5)


def make_pairs(lat: Lattice, mass: float, n: int, seed: int):
    """n pairs (b, x) with x white and b = M x (double precision operator),
    returned as float32 tensors (n, 3, V/2, 2)."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    B = torch.empty((n, 3, lat.Vh, 2), dtype=torch.float32, device="cuda")
    X = torch.empty_like(B)
    b64 = torch.empty((3, lat.Vh, 2), dtype=torch.float64, device="cuda")
    for k in range(n):
        x = _white((3, lat.Vh, 2), gen)
        lat.normal_op(mass, 0.0, x, out=b64)
        B[k].copy_(b64)
        X[k].copy_(x)
    return B, X


def solve_pairs(lat: Lattice, mass: float, n: int, seed: int, tol=1e-10):
    """n pairs with b white and x = M^-1 b from the double precision CG."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    B = torch.empty((n, 3, lat.Vh, 2), dtype=torch.float32, device="cuda")
    X = torch.empty_like(B)
    for k in range(n):
        b = _white((3, lat.Vh, 2), gen)
        x = torch.zeros_like(b)
        lat.cg(mass, 0.0, b, x, tol=tol)
        B[k].copy_(b)
        X[k].copy_(x)
    return B, X


# offsets of the parameter blocks in the network's weight vector (include/stag.h)
_W1S, _W1H, _W2, _WOUT = 0, 8, 72, 648


def polynomial_theta(c_self: float, c_dd: float, scale: float = 1.0):
    """Weights that make the network the fixed two-hop polynomial
    P = scale (c_self + c_dd D_eo D_oe), through channel 0.  With
    c_self = a + b - m^2 and c_dd = 1 it is P = scale (a + b - M): for a
    spectrum in [a, b] the preconditioned operator's condition number drops
    from b/a to (a + b)^2 / (4 a b)."""
    import numpy as np
    th = np.zeros(NET_NPARAM, np.complex128)
    th[_W1S] = 1.0
    for d in range(8):
        th[_W1H + d] = 0.5 if d < 4 else -0.5
        th[_W2 + 8 + 8 * d] = c_dd * (0.5 if d < 4 else -0.5)
    th[_W2] = c_self
    th[_WOUT] = scale
    return th


def lambda_max(lat: Lattice, mass: float, iters: int = 60, seed: int = 99) -> float:
    """Largest eigenvalue of M by power iteration with the library's operator."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    x = _white((3, lat.Vh, 2), gen)
    lam = 0.0
    for _ in range(iters):
        y = lat.normal_op(mass, 0.0, x)
        lam = float((x * y).sum() / (x * x).sum())
        x = y / torch.linalg.vector_norm(y)
    return lam


def save_params(path: str, net: Net, **meta):
    """The network's parameters (and any scalar metadata, e.g. the training
    loss) to an .npz file; read back with load_params (no pickled objects)."""
    import numpy as np
    np.savez(path, theta=net.get_params(), **{k: np.asarray(v) for k, v in meta.items()})


def load_params(path: str) -> Net:
    """A network with the parameters saved by save_params."""
    import numpy as np
    with np.load(path, allow_pickle=False) as f:
        return Net(f["theta"])


def init_theta(seed: int, scale: float = 0.1):
    import numpy as np
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(NET_NPARAM) + 1j * rng.standard_normal(NET_NPARAM))


def train(net: Net, data, steps: int, batch: int, lr: float, mode="bf16", seed: int = 0, log=None,
          plateau=None):
    """Adam on minibatches.  data: list of (Lattice, B, X); step k uses field
    k mod len(data) and a minibatch drawn from its pairs.  plateau =
    (window, rtol): stop early once the mean loss of the last `window` steps
    is less than rtol (relative) below the mean of the window before it.
    Returns the loss history (one value per step taken)."""
    gen = torch.Generator()
    gen.manual_seed(int(seed))
    losses = []
    t0 = time.perf_counter()
    for k in range(steps):
        lat, B, X = data[k % len(data)]
        n = B.shape[0]
        if batch >= n:
            b, x = B, X
        else:
            start = int(torch.randint(0, n - batch + 1, (1,), generator=gen))
            b, x = B[start:start + batch], X[start:start + batch]
        losses.append(net.train_step(lat, b, x, lr, mode))
        if log and (k + 1) % max(1, steps // 10) == 0:
            log(f"step {k + 1}/{steps} loss {losses[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
        if plateau and (k + 1) % plateau[0] == 0 and k + 1 >= 2 * plateau[0]:
            w = plateau[0]
            cur, prev = sum(losses[-w:]) / w, sum(losses[-2 * w:-w]) / w
            if prev - cur < plateau[1] * prev:
                if log:
                    log(f"plateau after {k + 1} steps: window mean {cur:.5f} against {prev:.5f}")
                break
    return losses


def compare(lat: Lattice, net: Net, mass: float, src: torch.Tensor, shift=0.0, tol=1e-10, max_iter=100000,
            modes=("bf16", "folded", "folded_bf16")):
    """Plain double precision CG against flexible CG with the network in
    each of `modes`, all from x = 0 on the same source: iterations, time and
    true residuals."""
    out = {}
    for name, n, mode in [("plain", None, "bf16")] + [(m, net, m) for m in modes]:
        x = torch.zeros_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rc, st = lat.fcg_solve(mass, shift, src, x, net=n, mode=mode, tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        out[name] = dict(status=rc, iters=st["iters"], seconds=time.perf_counter() - t0,
                         resid_true=st["resid_true"][0], fallback=st["fallback_used"])
    return out
