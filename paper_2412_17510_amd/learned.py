"""Training driver of the learned refinement preconditioner (network kernels in the HIP
library: mp_mpnn_* / mp_graph_*; this module only schedules calls).

Training data are pairs (r, e) with e = x* - x_k the error of the k-th iterate of a
plain DD CG solve of A x = A x* (x0 = 0) and r = A e (DD SpMV, leading component),
for a spread of k: the errors the inner solve meets once the rough components are
gone.  The loss of a pair is ||M r - e||_A^2 / ||e||_A^2, averaged over the pairs of
all training matrices; Adam on the float32 master weights (the network uses their
bfloat16 values).
"""
import numpy as np

from . import _binding as mp

SNAPSHOTS = (1, 2, 3, 5, 8, 12, 18, 27, 40, 60)


def init_params(seed, scale=0.1):
    """Small normal weights (std scale / sqrt(fan-in)), zero biases, float32."""
    rng = np.random.default_rng(seed)
    H, F = 64, 4
    parts = [rng.normal(0.0, scale / np.sqrt(F), (F, H)).ravel(), np.zeros(H)]
    for _ in range(3):
        parts += [rng.normal(0.0, scale / np.sqrt(H), H * H), rng.normal(0.0, scale / np.sqrt(H), H * H),
                  np.zeros(H)]
    parts += [rng.normal(0.0, scale / np.sqrt(H), H), np.zeros(1), rng.normal(0.0, scale / np.sqrt(H), H),
              np.zeros(1)]
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == mp.mp_mpnn_param_count()
    return theta


def cg_pairs(A, a, x_true, snapshots=SNAPSHOTS, plan=None):
    """(R, E): CUDA float64 tensors (len(snapshots), n) of residuals and errors of the
    DD CG iterates x_k (x0 = 0) for A x = b, b = A x_true."""
    import torch
    n = A.n_rows
    b = torch.empty((2, n), dtype=torch.float64, device="cuda")
    mp.mpspmv_csr_dd(A, a, x_true, b, plan=plan)
    E = torch.empty((len(snapshots), n), dtype=torch.float64, device="cuda")
    R = torch.empty_like(E)
    ev = torch.empty((2, n), dtype=torch.float64, device="cuda")
    rv = torch.empty((2, n), dtype=torch.float64, device="cuda")
    ws = mp._workspace(A, None)
    for i, k in enumerate(snapshots):
        x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
        mp.mpkrylov_cg(A, a, b, x, plan=plan, ws=ws, precond="jacobi", rtol=0.0, max_iter=k, check_every=k)
        mp.mpvec_dd_sub(x_true, x, ev)
        mp.mpspmv_csr_dd(A, a, ev, rv, plan=plan)
        E[i].copy_(ev[0])
        R[i].copy_(rv[0])
    return R, E


class Trainer:
    """Adam training of one network over a fixed set of matrices."""

    def __init__(self, theta0, lr=2e-3):
        self.net = mp.Mpnn()
        self.net.set_params(theta0)
        self.lr = lr
        self.step_count = 0
        self.items = []   # (graph, R, E)

    def add(self, A, a, R, E):
        self.items.append((mp.Graph(A, a), R, E))

    def step(self):
        """One Adam step on the mean loss over every pair; returns that mean loss."""
        self.net.zero_grads()
        total, count = 0.0, 0
        for g, R, E in self.items:
            losses = mp.mp_mpnn_loss_grad(self.net, g, R, E)
            total += float(losses.sum())
            count += losses.size
        self.step_count += 1
        self.net.adam_step(self.step_count, lr=self.lr, grad_scale=1.0 / count)
        return total / count

    def mean_loss(self):
        """Mean loss over every pair at the current parameters (gradients discarded)."""
        self.net.zero_grads()
        total, count = 0.0, 0
        for g, R, E in self.items:
            losses = mp.mp_mpnn_loss_grad(self.net, g, R, E)
            total += float(losses.sum())
            count += losses.size
        self.net.zero_grads()
        return total / count


def m_values(net, A, a):
    """M on A's pattern (CUDA float64 tensor of nnz values) from a trained network."""
    g = mp.Graph(A, a)
    out = mp.mp_mpnn_forward(net, g)
    import torch
    torch.cuda.synchronize()
    g.destroy()
    return out


def save(path, theta, **meta):
    np.savez(path, theta=np.asarray(theta, dtype=np.float32), **{k: np.asarray(v) for k, v in meta.items()})


def load(path):
    with np.load(path, allow_pickle=False) as f:
        return f["theta"].astype(np.float32)
