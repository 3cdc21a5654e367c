"""Shared helpers for the GPU parity tests (inputs to the device, error metrics)."""
import numpy as np
import torch

# Per-element normwise tolerance against the FP64 oracle:
#   max_ij |A_gpu - A_oracle| / max_ij |A_oracle|  <= TOL[precision]
# FP32 and FP16x2 meet 1e-5; BF16x2 (about 16 significant bits in G) is held to
# its stated bound 3e-5; BF16x3 (about 24 bits) to 1e-5.
TOL = {"fp32": 1e-5, "fp16x2": 1e-5, "bf16x2": 3e-5, "bf16x3": 1e-5}

# Adjoint: vertex gradients are sums of ~24 partially cancelling FP32 terms,
# judged against the sum of the norms of the incident elements' gradients (the
# normwise FP32 bound of the forward, per element);
# per-element coefficient gradients against the element's own scale.
TOL_VERTEX = 1e-5
TOL_COEFF = 1e-5
# Central differences of the oracle around a flattened tet (kappa ~ 3e3) carry
# their own truncation and cancellation error; the GPU is held to this looser
# bound only there, against the largest FD component.
TOL_FD_FLAT = 1e-4


def device():
    return torch.device("cuda", 0)


def mesh_to_device(mesh, dev=None):
    dev = dev or device()
    coords = torch.from_numpy(mesh.soa()).to(dev)
    conn = torch.from_numpy(np.ascontiguousarray(mesh.conn)).to(dev)
    return coords, conn


def vec_to_device(a, dev=None):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev or device())


def element_errors(A_gpu: np.ndarray, A_orc: np.ndarray) -> np.ndarray:
    """Normwise error of every element."""
    d = np.abs(A_gpu.astype(np.float64) - A_orc).reshape(len(A_orc), -1).max(axis=1)
    s = np.abs(A_orc).reshape(len(A_orc), -1).max(axis=1)
    return d / s


def vertex_scale(gvert: np.ndarray, conn: np.ndarray, n_vertices: int) -> np.ndarray:
    """Per vertex: the sum, over its incident elements, of that element's gradient
    norm (max over all its vertices and components of |per-element contribution|).

    Normwise per element, as the forward's element matrices are judged: an FP32
    element gradient is accurate relative to its largest entry, and the
    contribution to vertex 0 is minus the sum of the other columns of J-bar, so on
    a near-degenerate element it is a cancelled small difference of large
    numbers whose own magnitude is no scale for its rounding."""
    mag = np.abs(gvert).reshape(len(gvert), -1).max(axis=1)          # [E]
    s = np.zeros(n_vertices)
    np.add.at(s, conn.ravel(), np.repeat(mag, conn.shape[1]))
    return s
