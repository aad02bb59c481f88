"""FP64 CPU oracle for GSRF's data-parallel hot path (arXiv 2502.01826).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code, tables or constants generator
with the HIP path; both consume the seeded inputs of ``synth``.

It is the plain definition, not a fast method: every ray is tested against
every Gaussian in FP64, hits are taken in exact depth-key order, and the
complex front-to-back sum is formed with an explicit cumulative product.
Library primitives used as steps: matrix products, sort, cumprod, exp/sin/cos
and autograd (for gradients).

Paper passages followed (arXiv 2502.01826):
  * Gaussian primitive, Sigma = R S S^T R^T          -- Sec. 2 (3DGS preliminaries), Sec. 3.2
  * normalised Gaussian pdf at the chord midpoint    -- App. A.3 (discretized rendering), App. D.3
  * ray gamma(d) = r + d v, d >= r_rx                -- Sec. 3.3, eq. (ray definition)
  * spherical coordinates / 2D RF plane              -- Sec. 3.3, eqs. (spherical coords), (discretization)
  * Fourier-Legendre radiance                        -- Sec. 3.2, eq. (FLE)
  * complex ray-tracing sum                          -- Sec. 3.4, eq. (rendering); App. A
  * 3-sigma quadratic A d^2 + 2B d + (C-9) = 0        -- App. D.3.1-D.3.3
  * phase of a path of length d: 2 pi f d / c        -- Sec. 2 (RF propagation), worked example
  * single-antenna sum S_hat = sum_uv S_uv           -- Sec. 3.4 (loss, single antenna)
  * 64-bit splat key (tile | distance)               -- App. E (CUDA kernel paragraph)
  * paper footprint Sigma2D = J Sigma J^T,
    r_k = 3 sqrt(lambda_max), binning variant        -- Sec. 3.3 (splatting)

Readings taken where the paper is silent or ambiguous:
  R1  transmittance amplitude is 1 - o*G(x_mid) with o = sigmoid(logit); its
      phase is the free-space propagation term e^{-j 2 pi d / lambda}
      (App. A's continuous model with beta = 2 pi / lambda).
  R2  emission weight is the normalised pdf N*G (no opacity factor).
  R3  ellipsoid level 9 (3 sigma); R4 x_rep is the chord midpoint t = -B/A.
  R5  a Gaussian is hit iff B^2 - A(C-9) >= 0 and t = -B/A >= r_rx.
  R6  depth order is the per-Gaussian key bits(fp32(||mu-r||^2)), ties by
      Gaussian index; D^2 = (dx*dx + dy*dy) + dz*dz in FP64 without FMA.
  R8  rays sit at cell centres: alpha_u = 2 pi (u+1/2)/n_az,
      beta_v = el_lo + (el_hi-el_lo)(v+1/2)/n_el; the FP32-rounded unit
      vector is the ray direction for both sides.
  R10-R13 FLE: triangular |m| <= l <= L, K=(L+1)^2, index l^2+l+m,
      argument x = sin(elevation), unnormalised P_l^m with the
      Condon-Shortley phase, evaluated per ray.
  R14 path length d = ||mu - tx|| + t; no 1/d amplitude term.
  R15 c = 3e8 m/s; R16 stop before a hit whose T < t_min, alpha <= alpha_max.
  R17 RSSI = 10 log10 |sum_uv S_uv|^2.
  R25 binning culls with the bounding-sphere cap of radius 3*max(s) (exactly
      conservative), widened by 1e-5 rad.
  R28 at FP32-marginal discrete decisions both outcomes are correct.

Paper-literal variants, selected by grid attributes (0 = the readings above):
  depth_order = 1   each ray takes its hits in increasing chord-midpoint
                    parameter t_mid (App. A.3), ties by depth key then index;
  fle_eval = 1      the radiance psi_k is the FLE evaluated once per Gaussian
                    at the direction of mu_k from the receiver (the R13
                    alternative) instead of at the ray's direction;
  transmittance = 1 the transmittance of a hit is the chord form
                    rho = exp(-alpha_k dt) of App. A.2, dt = t_out - t_in the
                    3-sigma chord, with the amplitude attenuation coefficient
                    alpha_k = exp(logit) (per metre, >= 0), no excess phase
                    (the propagation phase of the path is kept, R1, R14) and no
                    opacity clamp.

Parity pinning: every function here is pinned by a CPU test in
tests/test_oracle_*.py against closed forms, library routines, the paper's
worked example or brute force.  The FLE conventions (R10-R13), the phase
convention (R14) and RSSI (R17) are readings: their numerical conventions are
pinned only up to the reading (closed forms of the chosen convention): parity
unpinned by the paper for those conventions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

C0 = 3.0e8          # m/s, R15 (the worked example in Sec. 2 needs exactly this)
LEVEL = 9.0         # 3-sigma Mahalanobis level, R3
CAP_SLACK = 1e-5    # rad, widening of the binning cap (R25)

F64 = torch.float64


def _f32(x: float) -> float:
    """Round a Python float to FP32 (the C ABI carries grid constants as float)."""
    return float(np.float32(x))


@dataclass
class Params:
    """FP64 torch view of one scene (inputs are promoted exactly from FP32)."""

    mu: torch.Tensor       # [N,3]
    log_s: torch.Tensor    # [N,3]
    q: torch.Tensor        # [N,4] (w,x,y,z), not necessarily unit
    a: torch.Tensor        # [N]
    c: torch.Tensor        # [N,K,2]

    @staticmethod
    def from_scene(scene, requires_grad: bool = False) -> "Params":
        t = lambda x: torch.tensor(np.asarray(x, dtype=np.float64), dtype=F64, requires_grad=requires_grad)
        return Params(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.logits), t(scene.coeffs))

    @property
    def n(self) -> int:
        return int(self.mu.shape[0])

    def tensors(self):
        return [self.mu, self.log_s, self.q, self.a, self.c]


# --------------------------------------------------------------------------
# a1: per-Gaussian activation (Sec. 2 3DGS preliminaries; App. B covariance
#     factorisation; App. A.3 normalised pdf)
# --------------------------------------------------------------------------

def rotation_matrix(q: torch.Tensor) -> torch.Tensor:
    """Unit-quaternion (w,x,y,z) rotation matrix; q is normalised first (R19)."""
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    R = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], dim=-1)
    return R.reshape(q.shape[:-1] + (3, 3))


def activate(P: Params):
    """Return (M = Sigma^-1, pdf normaliser N, opacity o) per Gaussian.

    Sigma = R S S^T R^T with S = diag(exp(log_s)), so Sigma^-1 = R diag(s^-2) R^T
    and |Sigma|^(1/2) = s1 s2 s3; N = (2 pi)^(-3/2) |Sigma|^(-1/2).
    """
    R = rotation_matrix(P.q)
    inv_s2 = torch.exp(-2.0 * P.log_s)
    M = R @ torch.diag_embed(inv_s2) @ R.transpose(-1, -2)
    Nn = (2.0 * math.pi) ** -1.5 * torch.exp(-P.log_s.sum(-1))
    o = torch.sigmoid(P.a)
    return M, Nn, o


# --------------------------------------------------------------------------
# Rays and the FLE basis (Sec. 3.3 spherical coordinates; Sec. 3.2 eq. FLE)
# --------------------------------------------------------------------------

def ray_angles(grid):
    """Cell-centre azimuth alpha_u and elevation beta_v in FP64 (R8)."""
    el_lo, el_hi = _f32(grid.el_lo), _f32(grid.el_hi)
    u = np.arange(grid.n_az, dtype=np.float64)
    v = np.arange(grid.n_el, dtype=np.float64)
    alpha = 2.0 * math.pi * (u + 0.5) / grid.n_az
    beta = el_lo + (el_hi - el_lo) * (v + 0.5) / grid.n_el
    return alpha, beta


def ray_dirs(grid) -> np.ndarray:
    """[n_el, n_az, 3] ray directions: FP64 unit vectors rounded to FP32 (R8)."""
    alpha, beta = ray_angles(grid)
    A, Bt = np.meshgrid(alpha, beta)            # [n_el, n_az]
    d = np.stack([np.cos(Bt) * np.cos(A), np.cos(Bt) * np.sin(A), np.sin(Bt)], axis=-1)
    return d.astype(np.float32).astype(np.float64)


def assoc_legendre(l: int, m: int, x):
    """Unnormalised associated Legendre P_l^m(x) with the Condon-Shortley phase (R12).

    Textbook recurrences: P_m^m = (-1)^m (2m-1)!! (1-x^2)^(m/2),
    P_{m+1}^m = x (2m+1) P_m^m, (l-m) P_l^m = (2l-1) x P_{l-1}^m - (l+m-1) P_{l-2}^m,
    and P_l^{-m} = (-1)^m (l-m)!/(l+m)! P_l^m.
    """
    x = np.asarray(x, dtype=np.float64)
    if m < 0:
        mm = -m
        return ((-1) ** mm) * math.factorial(l - mm) / math.factorial(l + mm) * assoc_legendre(l, mm, x)
    if m > l:
        return np.zeros_like(x)
    pmm = np.ones_like(x)
    if m > 0:
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        pmm = ((-1) ** m) * dfact * (1.0 - x * x) ** (m / 2.0)
    if l == m:
        return pmm
    pm1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pm1
    p_prev2, p_prev1 = pmm, pm1
    for ll in range(m + 2, l + 1):
        p = ((2 * ll - 1) * x * p_prev1 - (ll + m - 1) * p_prev2) / (ll - m)
        p_prev2, p_prev1 = p_prev1, p
    return p_prev1


def fle_basis(L: int, alpha, x) -> np.ndarray:
    """Y_i(alpha, x) = e^{j m alpha} P_l^m(x), i = l^2 + l + m; shape [..., (L+1)^2] complex128."""
    alpha = np.asarray(alpha, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(np.broadcast(alpha, x).shape + ((L + 1) ** 2,), dtype=np.complex128)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            out[..., l * l + l + m] = np.exp(1j * m * alpha) * assoc_legendre(l, m, x)
    return out


def fle_basis_dir(L: int, e: torch.Tensor):
    """FLE basis Y_i at unit directions e [n,3] (torch, differentiable): (Yr, Yi) [n, K].

    With w = e_x + j e_y = rho e^{j alpha} and x = e_z (rho^2 = 1 - x^2),
    e^{j m alpha} P_l^m(x) = w^m Q_l^m(x) where Q_l^m = P_l^m / (1 - x^2)^{m/2}
    follows the same textbook recurrences with Q_m^m = (-1)^m (2m-1)!!;
    m < 0 by P_l^{-m} = (-1)^m (l-m)!/(l+m)! P_l^m, so Y_{l,-m} =
    (-1)^m (l-m)!/(l+m)! conj(w)^m Q_l^m.  Smooth at the poles (no angle).
    """
    ex, ey, x = e[:, 0], e[:, 1], e[:, 2]
    K = (L + 1) ** 2
    wr = [torch.ones_like(x)]
    wi = [torch.zeros_like(x)]
    for m in range(1, L + 1):                                   # w^m by repeated products
        wr.append(wr[-1] * ex - wi[-1] * ey)
        wi.append(wr[-2] * ey + wi[-1] * ex)
    Yr = [None] * K
    Yi = [None] * K
    for m in range(0, L + 1):
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        q_prev2 = None
        q_prev1 = ((-1) ** m) * dfact * torch.ones_like(x)      # Q_m^m
        for l in range(m, L + 1):
            if l == m:
                q = q_prev1
            elif l == m + 1:
                q = x * (2 * m + 1) * q_prev1
                q_prev2, q_prev1 = q_prev1, q
            else:
                q = ((2 * l - 1) * x * q_prev1 - (l + m - 1) * q_prev2) / (l - m)
                q_prev2, q_prev1 = q_prev1, q
            Yr[l * l + l + m] = wr[m] * q
            Yi[l * l + l + m] = wi[m] * q
            if m > 0:
                f = ((-1) ** m) * math.factorial(l - m) / math.factorial(l + m)
                Yr[l * l + l - m] = f * wr[m] * q
                Yi[l * l + l - m] = -f * wi[m] * q
    return torch.stack(Yr, dim=-1), torch.stack(Yi, dim=-1)


def ray_basis(grid) -> np.ndarray:
    """[n_el, n_az, K] FLE basis at every ray: alpha_u and x = sin(beta_v) (R11)."""
    alpha, beta = ray_angles(grid)
    A, Bt = np.meshgrid(alpha, beta)
    return fle_basis(grid.fle_L, A, np.sin(Bt))


# --------------------------------------------------------------------------
# Depth keys (App. E 64-bit key; R6)
# --------------------------------------------------------------------------

def depth_key32(means, rx) -> np.ndarray:
    """bits(fp32(D^2)) with D^2 = (dx*dx + dy*dy) + dz*dz in FP64 (no FMA), d = mu - r."""
    mu = np.asarray(means, dtype=np.float64)
    r = np.asarray(rx, dtype=np.float64)
    d = mu - r
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    return d2.astype(np.float32).view(np.uint32).astype(np.int64)


def depth_order(means, rx) -> np.ndarray:
    """Gaussian indices sorted by (key32, index)."""
    k = depth_key32(means, rx)
    return np.argsort((k << 32) | np.arange(k.shape[0], dtype=np.int64), kind="stable")


# --------------------------------------------------------------------------
# a5/a6: complex front-to-back ray tracing (Sec. 3.4 eq. rendering, App. A, App. D.3)
# --------------------------------------------------------------------------

@dataclass
class Bands:
    """Widths of the FP32-marginal bands for discrete decisions (R28)."""

    q: float = 3e-4        # |Q - 9| (absolute, Mahalanobis^2 units)
    t: float = 1e-5        # |t - r_rx| relative to max(1, t)
    T: float = 3e-4        # |T - t_min| relative to t_min
    tie: float = 1e-6      # depth_order = 1: |t_i - t_j| of neighbouring hits (absolute, metres)


def _per_ray_terms(P: Params, act, rx, tx, lam, grid, dirs, Y, cols):
    """All per-(ray, Gaussian) quantities for Gaussians ``cols`` (in the given order).

    Follows App. D.3: delta = r - mu, A = v^T M v, B = v^T M delta,
    C = delta^T M delta, roots (-B +- sqrt(B^2 - A(C-9)))/A, midpoint t = -B/A,
    Mahalanobis^2 at the midpoint Q = C - B^2/A, pdf p = N exp(-Q/2).
    """
    M, Nn, o = act
    M, Nn, o = M[cols], Nn[cols], o[cols]
    mu = P.mu[cols]
    chord = getattr(grid, "transmittance", 0) == 1
    fle_g = getattr(grid, "fle_eval", 0) == 1
    R = dirs.shape[0]
    delta = rx[None, :] - mu                                   # [n,3]
    Md = (M @ delta.unsqueeze(-1)).squeeze(-1)                 # [n,3]
    C = (delta * Md).sum(-1)                                   # [n]
    vv = (dirs[:, :, None] * dirs[:, None, :]).reshape(R, 9)   # [R,9]
    A = vv @ M.reshape(-1, 9).T                                # [R,n]
    B = dirs @ Md.T                                            # [R,n]
    disc = B * B - A * (C[None, :] - LEVEL)
    t = -B / A
    Q = C[None, :] - B * B / A
    G = torch.exp(-0.5 * Q)
    p = Nn[None, :] * G
    if chord:
        # App. A.2: rho = exp(-alpha_k dt), dt = t_out - t_in = 2 sqrt(disc) / A
        with torch.no_grad():
            inside = disc > 0
        dt = torch.where(inside, 2.0 * torch.sqrt(torch.where(inside, disc, torch.ones_like(disc))) / A,
                         torch.zeros_like(disc))
        keep = torch.exp(-torch.exp(P.a[cols])[None, :] * dt)
        alpha = 1.0 - keep
    else:
        alpha = torch.clamp(o[None, :] * G, max=_f32(grid.alpha_max))
        keep = None
    dtx = torch.linalg.norm(mu - tx[None, :], dim=-1)          # ||mu - tx||
    d = dtx[None, :] + t                                       # path length (R14)
    phase = 2.0 * math.pi * d / lam
    c = P.c[cols]                                              # [n,K,2]
    if fle_g:
        # psi_k at the direction of mu_k from the receiver, one value per Gaussian
        e = mu - rx[None, :]
        e = e / torch.linalg.norm(e, dim=-1, keepdim=True)
        gYr, gYi = fle_basis_dir(grid.fle_L, e)                # [n,K]
        psi_r = ((gYr * c[:, :, 0]) - (gYi * c[:, :, 1])).sum(-1)[None, :].expand(R, -1)
        psi_i = ((gYi * c[:, :, 0]) + (gYr * c[:, :, 1])).sum(-1)[None, :].expand(R, -1)
    else:
        Yr, Yi = Y.real, Y.imag                                # [R,K]
        psi_r = Yr @ c[:, :, 0].T - Yi @ c[:, :, 1].T          # [R,n]
        psi_i = Yi @ c[:, :, 0].T + Yr @ c[:, :, 1].T
    cs, sn = torch.cos(phase), torch.sin(phase)
    # c~ = p * psi * e^{-j phase}
    ct_r = p * (psi_r * cs + psi_i * sn)
    ct_i = p * (psi_i * cs - psi_r * sn)
    out = dict(disc=disc, t=t, Q=Q, G=G, p=p, alpha=alpha, ct_r=ct_r, ct_i=ct_i)
    if keep is not None:
        out["keep"] = keep
    return out


def _order_by_tmid(terms, cols_t, grid):
    """depth_order = 1 (App. A.3): each ray's hits in increasing t_mid.

    Rows are permuted independently: hits first by t (stable, so equal t keep
    the depth-key order), then every non-hit in key order.  Returns the
    permuted terms and the [R, n] Gaussian ids per position."""
    r_rx = _f32(grid.r_rx)
    with torch.no_grad():
        hit = (terms["disc"] >= 0) & (terms["t"] >= r_rx)
        skey = torch.where(hit, terms["t"].detach(), torch.full_like(terms["t"], math.inf))
        perm = torch.sort(skey, dim=1, stable=True).indices
    out = {k: torch.gather(v, 1, perm) for k, v in terms.items()}
    return out, torch.gather(cols_t[None, :].expand(perm.shape[0], -1), 1, perm)


def _composite(terms, grid):
    """Front-to-back sum with termination; returns S (re, im), A_uv and masks."""
    r_rx, t_min = _f32(grid.r_rx), _f32(grid.t_min)
    with torch.no_grad():
        hit = (terms["disc"] >= 0) & (terms["t"] >= r_rx)
    if "keep" in terms:
        keep = torch.where(hit, terms["keep"], torch.ones_like(terms["keep"]))
    else:
        keep = 1.0 - torch.where(hit, terms["alpha"], torch.zeros_like(terms["alpha"]))
    incl = torch.cumprod(keep, dim=1)
    T = torch.cat([torch.ones_like(incl[:, :1]), incl[:, :-1]], dim=1)   # T before each Gaussian
    with torch.no_grad():
        active = hit & (T >= t_min)
    w = torch.where(active, T, torch.zeros_like(T))
    S_r = (w * terms["ct_r"]).sum(1)
    S_i = (w * terms["ct_i"]).sum(1)
    with torch.no_grad():
        A_uv = (w * torch.sqrt(terms["ct_r"] ** 2 + terms["ct_i"] ** 2)).sum(1)
    return S_r, S_i, A_uv, hit, active, T


def _pair_consts(pair):
    rx = torch.tensor(np.asarray(pair.rx, dtype=np.float64), dtype=F64)
    tx = torch.tensor(np.asarray(pair.tx, dtype=np.float64), dtype=F64)
    lam = C0 / float(pair.freq_hz)
    return rx, tx, lam


def _candidates(P, act, rx, grid, dirs, order, chunk_cols=65536):
    """Columns (in depth order) that pass the hit test for at least one ray (no grad)."""
    keep = []
    with torch.no_grad():
        for s in range(0, order.shape[0], chunk_cols):
            cols = order[s:s + chunk_cols]
            M = act[0][cols]
            delta = rx[None, :] - P.mu[cols].detach()
            Md = (M @ delta.unsqueeze(-1)).squeeze(-1)
            C = (delta * Md).sum(-1)
            R = dirs.shape[0]
            vv = (dirs[:, :, None] * dirs[:, None, :]).reshape(R, 9)
            A = vv @ M.reshape(-1, 9).T
            B = dirs @ Md.T
            disc = B * B - A * (C[None, :] - LEVEL)
            t = -B / A
            # keep marginal candidates too so that variants can be formed
            Q = C[None, :] - B * B / A
            near = ((disc >= 0) | (Q <= LEVEL + 0.01)) & (t >= _f32(grid.r_rx) * (1 - 1e-3))
            keep.append(cols[near.any(0).numpy()])
    return np.concatenate(keep) if keep else np.zeros(0, dtype=np.int64)


def trace(scene_or_params, pair, grid, rays_uv=None, *, grad=False, bands: Bands | None = None,
          ray_chunk: int = 64, rects=None):
    """Render rays (u, v) of one TX/RX pair.

    Returns a dict with S (complex128 [R]), A_uv (condition scale
    sum_i T_i |c~_i|, [R]), n_active [R], marginal [R] (bool), and, if
    ``grad``, the differentiable real/imag tensors S_r, S_i and the Params.
    ``rects`` (tu0, ntu, tv0, ntv, ...) restricts each ray to the Gaussians
    whose tile rectangle holds the ray's tile (a non-conservative binning).
    """
    P = scene_or_params if isinstance(scene_or_params, Params) else Params.from_scene(scene_or_params, grad)
    bands = bands or Bands()
    rx, tx, lam = _pair_consts(pair)
    if rays_uv is None:
        vv, uu = np.meshgrid(np.arange(grid.n_el), np.arange(grid.n_az), indexing="ij")
        rays_uv = np.stack([uu.ravel(), vv.ravel()], axis=1)
    rays_uv = np.asarray(rays_uv, dtype=np.int64).reshape(-1, 2)
    table = ray_dirs(grid)
    basis = ray_basis(grid)
    order = depth_order(P.mu.detach().numpy(), rx.numpy())
    act = activate(P)
    out_r, out_i, out_A, out_n, out_m, out_T, out_sig = [], [], [], [], [], [], []
    for s in range(0, rays_uv.shape[0], ray_chunk):
        uv = rays_uv[s:s + ray_chunk]
        dirs = torch.tensor(table[uv[:, 1], uv[:, 0]], dtype=F64)
        Y = torch.tensor(basis[uv[:, 1], uv[:, 0]])
        if P.n == 0:
            z = torch.zeros(uv.shape[0], dtype=F64)
            out_r.append(z); out_i.append(z); out_A.append(z)
            out_n.append(torch.zeros(uv.shape[0], dtype=torch.int64))
            out_m.append(torch.zeros(uv.shape[0], dtype=torch.bool))
            out_T.append(torch.ones(uv.shape[0], dtype=F64)); out_sig.append(torch.zeros(uv.shape[0], dtype=F64))
            continue
        cols = _candidates(P, act, rx, grid, dirs, order)
        if cols.shape[0] == 0:
            z = torch.zeros(uv.shape[0], dtype=F64)
            out_r.append(z); out_i.append(z); out_A.append(z)
            out_n.append(torch.zeros(uv.shape[0], dtype=torch.int64))
            out_m.append(torch.zeros(uv.shape[0], dtype=torch.bool))
            out_T.append(torch.ones(uv.shape[0], dtype=F64)); out_sig.append(torch.zeros(uv.shape[0], dtype=F64))
            continue
        cols_t = torch.tensor(cols)
        terms = _per_ray_terms(P, act, rx, tx, lam, grid, dirs, Y, cols_t)
        if rects is not None:
            allow = torch.tensor(rect_allow(rects, grid, uv)[:, cols])
            terms["disc"] = torch.where(allow, terms["disc"], torch.full_like(terms["disc"], -math.inf))
        if getattr(grid, "depth_order", 0) == 1:
            terms, colmat = _order_by_tmid(terms, cols_t, grid)
        else:
            colmat = cols_t[None, :].expand(uv.shape[0], -1)
        S_r, S_i, A_uv, hit, active, T = _composite(terms, grid)
        out_r.append(S_r); out_i.append(S_i); out_A.append(A_uv)
        out_n.append(active.sum(1))
        out_m.append(_marginal(terms, hit, active, T, grid, bands))
        with torch.no_grad():
            a_act = torch.where(active, terms["alpha"], torch.zeros_like(T))
            out_T.append(torch.prod(1.0 - a_act, dim=1))
            sig = (active.to(F64) * (colmat.to(F64) + 1.0)).sum(1)
            out_sig.append(sig)
    S_r = torch.cat(out_r); S_i = torch.cat(out_i)
    res = dict(
        S=(S_r.detach().numpy() + 1j * S_i.detach().numpy()),
        A_uv=torch.cat(out_A).numpy(),
        n_active=torch.cat(out_n).numpy(),
        marginal=torch.cat(out_m).numpy(),
        T_end=torch.cat(out_T).numpy(),
        active_sig=torch.cat(out_sig).numpy(),
        rays_uv=rays_uv,
    )
    if grad:
        res.update(S_r=S_r, S_i=S_i, params=P)
    return res


def _marginal(terms, hit, active, T, grid, bands: Bands):
    """Rays with a discrete decision inside the FP32-marginal band (R28).

    Only decisions the ray actually reaches count: a Gaussian whose incoming
    transmittance is already clearly below t_min is never examined.
    """
    with torch.no_grad():
        r_rx, t_min = _f32(grid.r_rx), _f32(grid.t_min)
        Q, t = terms["Q"], terms["t"]
        reached = T >= t_min * (1.0 - bands.T)
        tb = bands.t * torch.clamp(t.abs(), min=1.0)
        q_edge = ((Q - LEVEL).abs() <= bands.q) & (t >= r_rx - tb)
        t_edge = ((t - r_rx).abs() <= tb) & (Q <= LEVEL + bands.q)
        near_hit = hit | q_edge | t_edge
        T_edge = near_hit & ((T - t_min).abs() <= bands.T * t_min)
        flag = ((q_edge | t_edge) & reached | T_edge).any(1)
        if getattr(grid, "depth_order", 0) == 1:
            # neighbouring hits (rows already in t order) whose t_mid nearly tie:
            # FP32 may order them either way
            both = hit[:, 1:] & hit[:, :-1] & reached[:, :-1]
            tie = (t[:, 1:] - t[:, :-1]).abs() <= bands.tie
            flag = flag | (both & tie).any(1)
        return flag


def ray_sequence(scene, pair, grid, u: int, v: int, *, direction=None, basis=None):
    """Per-ray detail in depth order: every Gaussian's Q, t, alpha and c~
    (with depth_order = 1: the ray's hits in t_mid order, then the rest).

    ``direction`` / ``basis`` override the grid's ray (used by the worked
    example, which needs an exactly unit direction).  Returns numpy arrays
    indexed in depth order plus ``order`` (Gaussian ids).
    """
    P = scene if isinstance(scene, Params) else Params.from_scene(scene)
    rx, tx, lam = _pair_consts(pair)
    d = ray_dirs(grid)[v, u] if direction is None else np.asarray(direction, dtype=np.float64)
    y = ray_basis(grid)[v, u] if basis is None else np.asarray(basis, dtype=np.complex128)
    dirs = torch.tensor(d[None, :], dtype=F64)
    Y = torch.tensor(y[None, :])
    order = depth_order(P.mu.detach().numpy(), rx.numpy())
    act = activate(P)
    with torch.no_grad():
        terms = _per_ray_terms(P, act, rx, tx, lam, grid, dirs, Y, torch.tensor(order))
        if getattr(grid, "depth_order", 0) == 1:
            terms, colmat = _order_by_tmid(terms, torch.tensor(order), grid)
            order = colmat[0].numpy()
        S_r, S_i, A_uv, hit, active, T = _composite(terms, grid)
    g = lambda k: terms[k][0].detach().numpy()
    return dict(order=order, Q=g("Q"), t=g("t"), alpha=g("alpha"), p=g("p"),
                ct=g("ct_r") + 1j * g("ct_i"), hit=hit[0].numpy(), active=active[0].numpy(),
                T=T[0].detach().numpy(), S=complex(S_r[0]) + 1j * float(S_i[0]), A_uv=float(A_uv[0]))


def ray_variants(scene, pair, grid, u: int, v: int, bands: Bands | None = None, max_flip: int = 8):
    """All FP32-admissible results for one ray (R28).

    Decisions inside the marginal bands (hit test edges, termination edge) are
    enumerated; the returned list holds S for every combination.  A ray with
    more than ``max_flip`` marginal hit decisions returns None.
    """
    bands = bands or Bands()
    sq = ray_sequence(scene, pair, grid, u, v)
    r_rx, t_min = _f32(grid.r_rx), _f32(grid.t_min)
    Q, t, alpha, ct = sq["Q"], sq["t"], sq["alpha"], sq["ct"]
    tb = bands.t * np.maximum(np.abs(t), 1.0)
    sure = (Q <= LEVEL - bands.q) & (t >= r_rx + tb)
    maybe = (~sure) & (Q <= LEVEL + bands.q) & (t >= r_rx - tb)
    idx = np.nonzero(sure | maybe)[0]
    flips = [i for i in idx if maybe[i]]
    tmid = getattr(grid, "depth_order", 0) == 1
    ties = []
    if tmid:
        # neighbours in t order whose t_mid nearly tie: either order is admissible
        by_t = sorted(idx, key=lambda i: (t[i], i))
        for a_, b_ in zip(by_t[:-1], by_t[1:]):
            if abs(t[b_] - t[a_]) <= bands.tie:
                ties.append((a_, b_))
    if len(flips) + len(ties) > max_flip:
        return None
    out = []
    for mask in range(1 << (len(flips) + len(ties))):
        chosen = set(i for i in idx if sure[i])
        for b, i in enumerate(flips):
            if mask >> b & 1:
                chosen.add(i)
        seq = [i for i in idx if i in chosen]
        if tmid:
            seq = sorted(seq, key=lambda i: (t[i], i))
            for b, (a_, b_) in enumerate(ties):
                if mask >> (len(flips) + b) & 1 and a_ in chosen and b_ in chosen:
                    ia, ib = seq.index(a_), seq.index(b_)
                    seq[ia], seq[ib] = seq[ib], seq[ia]
        for thr in (t_min * (1 - bands.T), t_min, t_min * (1 + bands.T)):
            T, S = 1.0, 0.0 + 0.0j
            for i in seq:
                if T < thr:
                    break
                S += T * ct[i]
                T *= (1.0 - alpha[i])
            out.append(S)
    return out


def render(scene, pair, grid, **kw):
    """Full-grid render: S as complex128 [n_el, n_az] plus the per-ray diagnostics."""
    res = trace(scene, pair, grid, None, **kw)
    res["S_grid"] = res["S"].reshape(grid.n_el, grid.n_az)
    res["S_sum"] = res["S"].sum()
    return res


def rssi_dbm(S_sum) -> float:
    """Coherent single-antenna power 10 log10 |sum S_uv|^2 (R17); -inf for an empty scene."""
    p = abs(complex(S_sum)) ** 2
    return 10.0 * math.log10(p) if p > 0 else -math.inf


# --------------------------------------------------------------------------
# a7/a8: gradients = autograd of the plain definition (App. D; R21, R22)
# --------------------------------------------------------------------------

def vjp(scene, pair, grid, G, g_sum=None, rays_uv=None, ray_chunk: int = 64, rects=None):
    """Gradient of L = sum_r Re(conj(G_r + g_sum) S_r) w.r.t. the scene parameters.

    ``G`` is [R,2] (re, im) aligned with ``rays_uv`` (all rays when None);
    ``g_sum`` is the [2] cotangent of S_hat = sum over the listed rays.
    ``rects`` restricts the rays as in ``trace``.
    Returns FP64 numpy gradients keyed means/log_scales/quats/logits/coeffs.
    """
    P = Params.from_scene(scene, requires_grad=True)
    G = np.asarray(G, dtype=np.float64).reshape(-1, 2)
    if g_sum is not None:
        G = G + np.asarray(g_sum, dtype=np.float64).reshape(1, 2)
    Gt = torch.tensor(G, dtype=F64)
    res = trace(P, pair, grid, rays_uv, grad=True, ray_chunk=ray_chunk, rects=rects)
    L = (Gt[:, 0] * res["S_r"] + Gt[:, 1] * res["S_i"]).sum()
    if L.requires_grad:
        grads = torch.autograd.grad(L, P.tensors(), allow_unused=True)
    else:                                   # no ray hits anything: every gradient is zero
        grads = [None] * len(P.tensors())
    names = ["means", "log_scales", "quats", "logits", "coeffs"]
    out = {}
    for nm, g, t in zip(names, grads, P.tensors()):
        out[nm] = (torch.zeros_like(t) if g is None else g).detach().numpy()
    return out


def vjp_abs(scene, pair, grid, G, g_sum=None, rays_uv=None, ray_chunk: int = 4, rects=None):
    """``vjp`` together with an absolute scale of each gradient entry.

    Each gradient entry is dL/dtheta = Re(conj(G) dS/dtheta) summed over rays
    (R21).  Its scale is the sum over groups of ``ray_chunk`` rays of the
    group's complex magnitude |sum_r conj(G_r) dS_r/dtheta|, formed from the
    gradients for the cotangents G and j G (the second gives the imaginary
    part), so it does not vanish when the real projection happens to be small
    and it bounds |dL/dtheta|.  With one ray per group it is
    sum_r |G_r| |dS_r/dtheta|: what an FP32 evaluation of those terms, each with
    a small relative error, can be compared against, the way A_uv is for a ray.
    Returns (grads, scales), both keyed as vjp.
    """
    G = np.asarray(G, dtype=np.float64).reshape(-1, 2)
    if g_sum is not None:
        G = G + np.asarray(g_sum, dtype=np.float64).reshape(1, 2)
    jG = np.stack([-G[:, 1], G[:, 0]], axis=1)          # j (Gr + j Gi) = -Gi + j Gr
    if rays_uv is None:
        vv, uu = np.meshgrid(np.arange(grid.n_el), np.arange(grid.n_az), indexing="ij")
        rays_uv = np.stack([uu.ravel(), vv.ravel()], axis=1)
    rays_uv = np.asarray(rays_uv, dtype=np.int64).reshape(-1, 2)
    names = ["means", "log_scales", "quats", "logits", "coeffs"]
    tot = {nm: np.zeros(np.shape(getattr(scene, nm)), np.float64) for nm in names}
    scl = {nm: np.zeros(np.shape(getattr(scene, nm)), np.float64) for nm in names}
    for s in range(0, rays_uv.shape[0], ray_chunk):
        uv = rays_uv[s:s + ray_chunk]
        re = vjp(scene, pair, grid, G[s:s + ray_chunk], rays_uv=uv, ray_chunk=ray_chunk, rects=rects)
        im = vjp(scene, pair, grid, jG[s:s + ray_chunk], rays_uv=uv, ray_chunk=ray_chunk, rects=rects)
        for nm in names:
            tot[nm] += re[nm]
            scl[nm] += np.hypot(re[nm], im[nm])
    return tot, scl


# --------------------------------------------------------------------------
# a2/a3/a4: binning definition -- conservative cap rectangle and tile lists
# (Sec. 3.3 splatting; App. E grids of 16x16 rays and 64-bit keys; R25)
# --------------------------------------------------------------------------

def _near_int(x, tol=1e-9):
    x = np.asarray(x, dtype=np.float64)
    return np.abs(x - np.round(x)) <= tol * np.maximum(1.0, np.abs(x))


def cap_rects(means, log_scales, rx, grid):
    """Tile rectangle covered by each Gaussian's bounding cap, FP64.

    Returns int64 arrays (tu0, ntu, tv0, ntv) -- ntu*ntv = 0 means culled;
    azimuth tiles run tu0, tu0+1, ... modulo the tile-column count -- and a
    bool array ``marginal`` flagging Gaussians where a rounding decision sat
    within 1e-9 of its threshold (both outcomes then count as correct).

    Definition: e = mu - r, D = |e|, Rb = 3 max(s).  Culled if
    D + Rb < r_rx (1 - 1e-6).  If D <= Rb (1 + 1e-6) every ray row and column
    is covered.  Otherwise the cap half-angle is theta = asin(Rb/D) + 1e-5
    around elevation beta_c = atan2(e_z, |e_xy|) and azimuth
    alpha_c = atan2(e_y, e_x); the rows whose centre elevation lies in
    [beta_c - theta, beta_c + theta] are covered; if that band reaches a pole
    every column is covered, else the columns whose centre azimuth lies within
    asin(sin theta / cos beta_c) of alpha_c (modulo 2 pi).
    """
    mu = np.asarray(means, dtype=np.float64)
    r = np.asarray(rx, dtype=np.float64)
    ls = np.asarray(log_scales, dtype=np.float64)
    n = mu.shape[0]
    n_az, n_el, tw, th = grid.n_az, grid.n_el, grid.tile_w, grid.tile_h
    nta = -(-n_az // tw)
    el_lo, el_hi, r_rx = _f32(grid.el_lo), _f32(grid.el_hi), _f32(grid.r_rx)
    e = mu - r
    D2 = (e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2]
    D = np.sqrt(D2)
    Rb = 3.0 * np.exp(np.max(ls, axis=1)) if n else np.zeros(0)
    cull_r = D + Rb < r_rx * (1.0 - 1e-6)
    inside = D <= Rb * (1.0 + 1e-6)
    marg = np.zeros(n, dtype=bool)
    marg |= np.abs((D + Rb) - r_rx * (1.0 - 1e-6)) <= 1e-12 * np.maximum(1.0, D)
    marg |= np.abs(D - Rb * (1.0 + 1e-6)) <= 1e-12 * np.maximum(1.0, D)
    dbeta = (el_hi - el_lo) / n_el
    dalpha = 2.0 * math.pi / n_az
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(inside, 0.0, Rb / np.where(D > 0, D, 1.0))
        theta = np.arcsin(np.minimum(ratio, 1.0)) + CAP_SLACK
        bc = np.arctan2(e[:, 2], np.sqrt(e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]))
        lo, hi = bc - theta, bc + theta
        xv_lo = (lo - el_lo) / dbeta - 0.5
        xv_hi = (hi - el_lo) / dbeta - 0.5
        v_lo = np.ceil(xv_lo)
        v_hi = np.floor(xv_hi)
        marg |= (~inside) & (_near_int(xv_lo) | _near_int(xv_hi))
        v_lo = np.where(inside, 0, np.maximum(v_lo, 0))
        v_hi = np.where(inside, n_el - 1, np.minimum(v_hi, n_el - 1))
        pole = inside | (hi >= math.pi / 2) | (lo <= -math.pi / 2)
        marg |= (~inside) & ((np.abs(hi - math.pi / 2) <= 1e-12) | (np.abs(lo + math.pi / 2) <= 1e-12))
        ac = np.arctan2(e[:, 1], e[:, 0])
        da = np.arcsin(np.minimum(np.sin(theta) / np.cos(bc), 1.0))
        xu_lo = (ac - da) / dalpha - 0.5
        xu_hi = (ac + da) / dalpha - 0.5
        u_lo = np.ceil(xu_lo)
        u_hi = np.floor(xu_hi)
        marg |= (~pole) & (_near_int(xu_lo) | _near_int(xu_hi))
    full = pole | ((u_hi - u_lo + 1) >= n_az)
    no_col = (~full) & (u_hi < u_lo)          # no column centre inside the cap
    u_lo = np.where(full | no_col, 0, u_lo)
    u_hi = np.where(no_col, 0, u_hi)
    u_hi = np.where(full, n_az - 1, u_hi)
    wrap_neg = u_lo < 0
    u_lo = np.where(wrap_neg, u_lo + n_az, u_lo).astype(np.int64)
    u_hi = np.where(wrap_neg, u_hi + n_az, u_hi).astype(np.int64)
    tu0 = u_lo // tw
    ntu = np.where(u_hi < n_az, u_hi // tw - tu0 + 1, (nta - tu0) + (u_hi - n_az) // tw + 1)
    over = ntu >= nta
    tu0 = np.where(over, 0, tu0)
    ntu = np.where(over, nta, ntu)
    v_lo = v_lo.astype(np.int64)
    v_hi = v_hi.astype(np.int64)
    tv0 = v_lo // th
    ntv = v_hi // th - tv0 + 1
    visible = (~cull_r) & (v_lo <= v_hi) & (~no_col)
    ntu = np.where(visible, ntu, 0)
    ntv = np.where(visible, ntv, 0)
    tu0 = np.where(visible, tu0, 0)
    tv0 = np.where(visible, tv0, 0)
    return tu0, ntu, tv0, ntv, marg


def footprint_jacobian(e, grid):
    """Jacobian (2 x 3, ray-index units) of the map x -> (u, v) at offset e = x - r.

    u = alpha / d_alpha with alpha = atan2(e_y, e_x), v = (beta - el_lo) / d_beta
    with beta = atan2(e_z, |e_xy|) (Sec. 3.3, eqs. spherical coords and
    discretization).  Undefined on the vertical through the receiver.
    """
    ex, ey, ez = (float(c) for c in e)
    n_az, n_el = grid.n_az, grid.n_el
    dalpha = 2.0 * math.pi / n_az
    dbeta = (_f32(grid.el_hi) - _f32(grid.el_lo)) / n_el
    rho2 = ex * ex + ey * ey
    rho = math.sqrt(rho2)
    D2 = rho2 + ez * ez
    ja = np.array([-ey / rho2, ex / rho2, 0.0]) / dalpha
    jb = np.array([-ez * ex / (D2 * rho), -ez * ey / (D2 * rho), rho / D2]) / dbeta
    return np.stack([ja, jb])


def footprint_rects(means, log_scales, quats, rx, grid):
    """Tile rectangle of each Gaussian's paper footprint, FP64 (reading R25, variant).

    Sec. 3.3 (splatting): the projected centre (u_k, v_k) is the ray cell of
    the direction mu - r (spherical coordinates, then floor discretisation);
    Sigma2D = J Sigma J^T with J the Jacobian of that map at mu; the radius is
    r_k = 3 sqrt(lambda_max(Sigma2D)), and rays with
    (u - u_k)^2 + (v - v_k)^2 <= r_k^2 are the splat.  Binning keeps the
    circle's bounding square u_k +- m, v_k +- m, m = floor(r_k), rows clipped
    to the grid, columns modulo n_az.  Not conservative (J linearises the map).
    The cap's exact guards stay: culled if D + Rb < r_rx (1 - 1e-6), every ray
    covered if D <= Rb (1 + 1e-6) (Rb = 3 max s), every column covered on the
    receiver's vertical or when 2m + 1 >= n_az.

    Returns (tu0, ntu, tv0, ntv, marginal) like ``cap_rects``; marginal flags a
    floor within 1e-9 (relative) of an integer.
    """
    mu = np.asarray(means, dtype=np.float64)
    r = np.asarray(rx, dtype=np.float64)
    ls = np.asarray(log_scales, dtype=np.float64)
    R = rotation_matrix(torch.tensor(np.asarray(quats, dtype=np.float64))).numpy()
    n = mu.shape[0]
    n_az, n_el, tw, th = grid.n_az, grid.n_el, grid.tile_w, grid.tile_h
    nta = -(-n_az // tw)
    el_lo, el_hi, r_rx = _f32(grid.el_lo), _f32(grid.el_hi), _f32(grid.r_rx)
    dalpha = 2.0 * math.pi / n_az
    dbeta = (el_hi - el_lo) / n_el
    out = np.zeros((n, 4), dtype=np.int64)
    marg = np.zeros(n, dtype=bool)
    for g in range(n):
        e = mu[g] - r
        D = math.sqrt((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2])
        Rb = 3.0 * math.exp(ls[g].max())
        if D + Rb < r_rx * (1.0 - 1e-6):
            continue
        rho = math.hypot(e[0], e[1])
        if D <= Rb * (1.0 + 1e-6):
            v_lo, v_hi, u_lo, u_hi, full = 0, n_el - 1, 0, n_az - 1, True
        else:
            alpha = math.atan2(e[1], e[0])
            if alpha < 0:
                alpha += 2.0 * math.pi
            xu = alpha / dalpha
            xv = (math.atan2(e[2], rho) - el_lo) / dbeta
            u_k = min(math.floor(xu), n_az - 1)
            v_k = math.floor(xv)
            if rho == 0.0:
                m, full = n_el, True
                marg[g] |= bool(_near_int(xv))
            else:
                Sigma = R[g] @ np.diag(np.exp(2.0 * ls[g])) @ R[g].T
                J = footprint_jacobian(e, grid)
                S2 = J @ Sigma @ J.T
                a, b, c = S2[0, 0], S2[0, 1], S2[1, 1]
                lam_max = 0.5 * (a + c) + math.sqrt(0.25 * (a - c) ** 2 + b * b)
                r_k = 3.0 * math.sqrt(lam_max)
                m = math.floor(r_k) if r_k < 1e9 else 10 ** 9      # NaN or huge: every column
                full = 2 * m + 1 >= n_az
                marg[g] |= bool(_near_int(xu) | _near_int(xv) | _near_int(r_k))
            v_lo, v_hi = max(v_k - m, 0), min(v_k + m, n_el - 1)
            u_lo, u_hi = (0, n_az - 1) if full else (u_k - m, u_k + m)
        if v_lo > v_hi:
            continue
        if u_lo < 0:
            u_lo, u_hi = u_lo + n_az, u_hi + n_az
        tu0 = u_lo // tw
        ntu = u_hi // tw - tu0 + 1 if u_hi < n_az else (nta - tu0) + (u_hi - n_az) // tw + 1
        if ntu >= nta:
            tu0, ntu = 0, nta
        tv0 = v_lo // th
        out[g] = (tu0, ntu, tv0, v_hi // th - tv0 + 1)
    return out[:, 0], out[:, 1], out[:, 2], out[:, 3], marg


def rect_allow(rects, grid, rays_uv):
    """Per-(ray, Gaussian) mask: the ray's tile lies in the Gaussian's rectangle."""
    tu0, ntu, tv0, ntv = (np.asarray(x, dtype=np.int64) for x in rects[:4])
    nta = grid.n_tiles_az
    uv = np.asarray(rays_uv, dtype=np.int64).reshape(-1, 2)
    tu = (uv[:, 0] // grid.tile_w)[:, None]
    tv = (uv[:, 1] // grid.tile_h)[:, None]
    return ((ntu * ntv > 0)[None, :] & (tv >= tv0[None, :]) & (tv < (tv0 + ntv)[None, :])
            & (((tu - tu0[None, :]) % nta) < ntu[None, :]))


def rect_tiles(tu0, ntu, tv0, ntv, grid):
    """Tile ids (row-major over tile rows, tile columns) of one rectangle."""
    nta = grid.n_tiles_az
    out = []
    for tv in range(tv0, tv0 + ntv):
        for k in range(ntu):
            out.append(tv * nta + (tu0 + k) % nta)
    return out


def tile_lists(means, log_scales, rx, grid):
    """Per-tile Gaussian lists in (key32, index) order, plus per-tile keys.

    Returns (lists, keys, marginal) where lists[t] / keys[t] are int64 arrays
    and marginal is the per-Gaussian flag from ``cap_rects``.
    """
    tu0, ntu, tv0, ntv, marg = cap_rects(means, log_scales, rx, grid)
    key = depth_key32(means, rx)
    buckets = [[] for _ in range(grid.n_tiles)]
    for g in np.nonzero(ntu * ntv)[0]:
        for t in rect_tiles(int(tu0[g]), int(ntu[g]), int(tv0[g]), int(ntv[g]), grid):
            buckets[t].append(g)
    lists, keys = [], []
    for b in buckets:
        b = np.asarray(b, dtype=np.int64)
        if b.size:
            o = np.lexsort((b, key[b]))
            b = b[o]
        lists.append(b)
        keys.append(key[b] if b.size else np.zeros(0, dtype=np.int64))
    return lists, keys, marg
