"""Dense brute-force reference in float64 PyTorch (CPU), test-only.

Every Gaussian is evaluated at every pixel (no tiles, no lists); order is a
global sort by (fp32 depth, id); gradients come from autograd.  It exists to
pin the C oracle, so it is written independently of it: torch tensor algebra
for the projection, the Cartesian real-SH polynomials (rather than the
oracle's Legendre recurrence), and cumulative products for the transmittance.

Sec. 3.1 (splatting, alpha = o * G2D, depth order), Eq. (3)-(4) (masked
compositing) and the background term of the supplementary derivation.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def sh_cartesian(deg: int, d: torch.Tensor) -> torch.Tensor:
    """Real SH (no Condon-Shortley phase) of a unit direction d [N,3] -> [N,(deg+1)^2]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [torch.full_like(x, 0.5 * math.sqrt(1.0 / pi))]
    if deg >= 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [c1 * y, c1 * z, c1 * x]
    if deg >= 2:
        out += [0.5 * math.sqrt(15.0 / pi) * x * y,
                0.5 * math.sqrt(15.0 / pi) * y * z,
                0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0),
                0.5 * math.sqrt(15.0 / pi) * x * z,
                0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if deg >= 3:
        out += [0.25 * math.sqrt(35.0 / (2 * pi)) * y * (3.0 * x * x - y * y),
                0.5 * math.sqrt(105.0 / pi) * x * y * z,
                0.25 * math.sqrt(21.0 / (2 * pi)) * y * (5.0 * z * z - 1.0),
                0.25 * math.sqrt(7.0 / pi) * (5.0 * z ** 3 - 3.0 * z),
                0.25 * math.sqrt(21.0 / (2 * pi)) * x * (5.0 * z * z - 1.0),
                0.25 * math.sqrt(105.0 / pi) * (x * x - y * y) * z,
                0.25 * math.sqrt(35.0 / (2 * pi)) * x * (x * x - 3.0 * y * y)]
    return torch.stack(out, dim=1)


def quat_to_matrix(q: torch.Tensor) -> torch.Tensor:
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def params_from_scene(scene: dict, requires_grad: bool = True) -> dict:
    out = {}
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        out[k] = torch.tensor(np.asarray(scene[k], np.float64), requires_grad=requires_grad)
    return out


def project_dense(p: dict, cam: dict, st) -> dict:
    vm = torch.tensor(np.asarray(cam["viewmat"], np.float32).astype(np.float64))
    W, tv = vm[:3, :3], vm[:3, 3]
    fx, fy = float(cam["fx"]), float(cam["fy"])
    cx, cy = float(cam["cx"]), float(cam["cy"])
    t = p["means"] @ W.T + tv
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    depth32 = tz.detach().numpy().astype(np.float32)
    valid = torch.tensor(depth32.astype(np.float64) > float(np.float32(st.near_plane)))
    tzs = torch.where(valid, tz, torch.ones_like(tz))
    u = fx * tx / tzs + cx
    v = fy * ty / tzs + cy
    limx = float(np.float32(st.jac_clamp)) * 0.5 * cam["width"] / fx
    limy = float(np.float32(st.jac_clamp)) * 0.5 * cam["height"] / fy
    sx = torch.clamp(tx / tzs, -limx, limx)
    sy = torch.clamp(ty / tzs, -limy, limy)
    zero = torch.zeros_like(tzs)
    J = torch.stack([torch.stack([fx / tzs, zero, -fx * sx / tzs], 1),
                     torch.stack([zero, fy / tzs, -fy * sy / tzs], 1)], 1)
    R = quat_to_matrix(p["quats"])
    s2 = torch.exp(2.0 * p["log_scales"])
    Sigma3 = R @ torch.diag_embed(s2) @ R.transpose(1, 2)
    T = J @ W
    dil = float(np.float32(st.dilation))
    Sigma2 = T @ Sigma3 @ T.transpose(1, 2) + dil * torch.eye(2, dtype=torch.float64)
    a, b, c = Sigma2[:, 0, 0], Sigma2[:, 0, 1], Sigma2[:, 1, 1]
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], 1)
    campos = -(W.T @ tv)
    dv = p["means"] - campos
    dirs = dv / dv.norm(dim=1, keepdim=True)
    deg = st.sh_degree
    Y = sh_cartesian(deg, dirs)
    col = torch.einsum("nk,nkc->nc", Y, p["sh"]) + 0.5
    col = torch.clamp(col, min=0.0)
    opac = torch.sigmoid(p["opacity_logits"])
    return dict(u=u, v=v, conic=conic, color=col, opacity=opac, valid=valid & (det.detach() > 0),
                depth32=depth32)


def render_dense(p: dict, cam: dict, st, mask: torch.Tensor) -> tuple:
    """Image [3,H,W] and final transmittance [H,W] of one view."""
    pr = project_dense(p, cam, st)
    n = pr["u"].shape[0]
    order = np.lexsort((np.arange(n), pr["depth32"]))
    order = torch.tensor(order)
    H, Wd = cam["height"], cam["width"]
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64) + 0.5,
                            torch.arange(Wd, dtype=torch.float64) + 0.5, indexing="ij")
    px, py = xs.reshape(-1, 1), ys.reshape(-1, 1)
    u, v = pr["u"][order][None, :], pr["v"][order][None, :]
    conic = pr["conic"][order]
    dx, dy = u - px, v - py
    Q = conic[None, :, 0] * dx * dx + 2.0 * conic[None, :, 1] * dx * dy + conic[None, :, 2] * dy * dy
    G = torch.exp(-0.5 * Q)
    amax = float(np.float32(st.alpha_max))
    alpha = torch.clamp(pr["opacity"][order][None, :] * G, max=amax)
    if st.exact_mode:
        passes = torch.ones_like(alpha, dtype=torch.bool)
        tmin = 0.0
    else:
        amin = float(np.float32(st.alpha_min))
        passes = (Q.detach() <= float(np.float32(st.q_max))) & (alpha.detach() >= amin)
        tmin = float(np.float32(st.t_min))
    passes = passes & pr["valid"][order][None, :]
    Ma = mask[order][None, :] * alpha * passes
    one_minus = 1.0 - Ma
    Tincl = torch.cumprod(one_minus, dim=1)
    alive = Tincl.detach() >= tmin  # entry i kept iff T_{i+1} >= T_min
    Ma_alive = Ma * alive
    Tincl_alive = torch.cumprod(1.0 - Ma_alive, dim=1)
    Texcl = torch.cat([torch.ones_like(Tincl_alive[:, :1]), Tincl_alive[:, :-1]], dim=1)
    wgt = Ma_alive * Texcl
    col = pr["color"][order]
    C = wgt @ col
    Tfin = Tincl_alive[:, -1] if n > 0 else torch.ones(px.shape[0], dtype=torch.float64)
    bg = torch.tensor([float(np.float32(b)) for b in st.bg], dtype=torch.float64)
    C = C + Tfin[:, None] * bg[None, :]
    return C.T.reshape(3, H, Wd), Tfin.reshape(H, Wd)
