"""CPU FP64 oracle for Levenberg-Marquardt bundle adjustment.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the device library (no kernels, headers, helpers or tables); both consume the
same seeded arrays from ``synth``.

What it computes (paper: Sec. 4.3, Iterative Triangulation and Mapping):

* reprojection residual of point X_j in camera i, r = pi(K_i (R_i X_j + t_i)) - z
  (the reprojection-error equation of Sec. 4.3; the paper's equation indexes the
  camera by j, its text by i: here i is the camera and j the point);
* the robust objective of Sec. 4.3 restricted to its reprojection term,
  C = 1/2 sum_k rho(||r_k||^2) with rho Huber on the squared norm, or rho(s) = s;
* designated-fixed camera poses (Sec. 4.3), removed from the unknowns;
* optionally the prior terms of the Sec. 4.3 objective: the absolute pose
  constraint e_a = ||T_i - T_i,init||^2 (Eq. abs) and the sequential constraint
  e_c = ||T_i T_{i+k}^-1 - T_i,init T_{i+k,init}^-1||^2 (Eq. seq), read as squared
  Frobenius norms of the 3x4 upper parts, weighted by lambda_a and lambda_c and
  entering C with the same factor 1/2 as the reprojection term;
* pose-graph optimisation (Sec. 4.2): nodes are poses, edges (i, j) carry a
  measured relative pose M_ij and the error T_i T_j^-1 - M_ij, the form of the
  sequential and extrinsic constraints (Eq. seq, Eq. extrinsic) that loop-closure
  edges share; the objective sum e^T Omega e with Omega diagonal, one weight for
  the nine rotation entries and one for the three translation entries.  It is the
  same machinery as the sequential prior with explicit pairs, measurements and
  weights, and no observations (``pose_graph_problem``);
* vehicle-rig BA (Sec. 4.4): camera poses composed from shared camera-to-vehicle
  extrinsics and per-frame vehicle poses, both unknown, with the absolute prior on the
  extrinsics and the rigidity constraints of Eq. extrinsic (``RigProblem``, ``lm_rig``);
* Levenberg-Marquardt with Marquardt diagonal scaling and Nielsen's damping
  schedule (Madsen, Nielsen, Tingleff 2004, Sec. 3.2), left SE(3) increments;
* three solvers of the damped normal equations (H + lambda D) delta = -g:
  - ``lm_dense``: the full H from the sparse Jacobian, dense Cholesky;
  - ``lm_schur``: points eliminated (Triggs et al. 2000, Sec. 6.1), the reduced
    camera system solved exactly or by block-Jacobi preconditioned CG
    (Hestenes-Stiefel), then points back-substituted;
* ``pose_only_gn``: Gauss-Newton on one 6-DoF pose with the map fixed, the
  localization mode of Sec. 6.4.2.

Readings where the paper is silent (pose convention, loss form, damping, the
update map, PCG stopping rule, masking of points behind a camera) are the ones
listed in the design notes; each function states the reading it uses.

Parity pins: every function here is checked by ``tests/test_oracle_pins.py``
against closed forms, finite differences, SciPy routines or invariants.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg
import scipy.sparse as sp

Z_MIN = 1e-6          # depth (camera units) at or below which an observation is masked
LAMBDA_MIN = 1e-12
LAMBDA_MAX = 1e16
D_MIN = 1e-6
D_MAX = 1e32
ACCEPT_RHO = 1e-3

STATUS_OK = 0
STATUS_DAMPING = 1     # lambda reached its upper clamp
STATUS_NUMERICAL = 2   # non-finite cost


# ----------------------------------------------------------------------------- geometry

def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z) -> rotation matrix (Hamilton convention).
    The quaternion is normalised first."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def hat(v: np.ndarray) -> np.ndarray:
    """Skew matrix [v]x with [v]x a = v x a."""
    v = np.asarray(v, dtype=np.float64)
    M = np.zeros(v.shape[:-1] + (3, 3))
    M[..., 0, 1] = -v[..., 2]
    M[..., 0, 2] = v[..., 1]
    M[..., 1, 0] = v[..., 2]
    M[..., 1, 2] = -v[..., 0]
    M[..., 2, 0] = -v[..., 1]
    M[..., 2, 1] = v[..., 0]
    return M


def se3_exp(xi: np.ndarray):
    """Exponential map of se(3), xi = (rho, phi) with rho the translational and phi
    the rotational part.  Returns (R, t) with R = exp([phi]x) (Rodrigues) and
    t = V(phi) rho, V = I + B [phi]x + C [phi]x^2, A = sin(th)/th,
    B = (1 - cos th)/th^2, C = (th - sin th)/th^3.  Series in th^2 below 1e-4."""
    xi = np.asarray(xi, dtype=np.float64)
    rho = xi[..., 0:3]
    phi = xi[..., 3:6]
    th2 = np.sum(phi * phi, axis=-1)
    th = np.sqrt(th2)
    small = th < 1e-4
    ths = np.where(small, 1.0, th)
    A = np.where(small, 1 - th2 / 6 + th2 * th2 / 120, np.sin(ths) / ths)
    # (1 - cos th) / th^2 written with the half-angle identity 1 - cos th = 2 sin^2(th/2),
    # which avoids the cancellation of 1 - cos th for small th
    sh = np.sin(0.5 * ths) / (0.5 * ths)
    B = np.where(small, 0.5 - th2 / 24 + th2 * th2 / 720, 0.5 * sh * sh)
    Cc = np.where(small, 1.0 / 6 - th2 / 120 + th2 * th2 / 5040,
                  (ths - np.sin(ths)) / (ths * ths * ths))
    K = hat(phi)
    K2 = K @ K
    eye = np.broadcast_to(np.eye(3), K.shape)
    R = eye + A[..., None, None] * K + B[..., None, None] * K2
    V = eye + B[..., None, None] * K + Cc[..., None, None] * K2
    t = np.einsum("...ij,...j->...i", V, rho)
    return R, t


def rot_to_quat(R: np.ndarray) -> np.ndarray:
    """Rotation matrix -> unit quaternion (w, x, y, z) with w >= 0 (Shepperd 1978)."""
    R = np.asarray(R, dtype=np.float64)
    flat = R.reshape(-1, 3, 3)
    out = np.empty((flat.shape[0], 4))
    for n, M in enumerate(flat):
        tr = M[0, 0] + M[1, 1] + M[2, 2]
        cands = [tr, M[0, 0], M[1, 1], M[2, 2]]
        k = int(np.argmax(cands))
        if k == 0:
            s = math.sqrt(1.0 + tr) * 2
            q = [0.25 * s, (M[2, 1] - M[1, 2]) / s, (M[0, 2] - M[2, 0]) / s, (M[1, 0] - M[0, 1]) / s]
        elif k == 1:
            s = math.sqrt(1.0 + M[0, 0] - M[1, 1] - M[2, 2]) * 2
            q = [(M[2, 1] - M[1, 2]) / s, 0.25 * s, (M[0, 1] + M[1, 0]) / s, (M[0, 2] + M[2, 0]) / s]
        elif k == 2:
            s = math.sqrt(1.0 + M[1, 1] - M[0, 0] - M[2, 2]) * 2
            q = [(M[0, 2] - M[2, 0]) / s, (M[0, 1] + M[1, 0]) / s, 0.25 * s, (M[1, 2] + M[2, 1]) / s]
        else:
            s = math.sqrt(1.0 + M[2, 2] - M[0, 0] - M[1, 1]) * 2
            q = [(M[1, 0] - M[0, 1]) / s, (M[0, 2] + M[2, 0]) / s, (M[1, 2] + M[2, 1]) / s, 0.25 * s]
        q = np.array(q)
        q /= np.linalg.norm(q)
        if q[0] < 0:
            q = -q
        out[n] = q
    return out.reshape(R.shape[:-2] + (4,))


# ----------------------------------------------------------------------------- residual & loss

def project(K: np.ndarray, R: np.ndarray, t: np.ndarray, X: np.ndarray):
    """Perspective projection of the reprojection-error equation (Sec. 4.3):
    P_c = R X + t, u = fx x/z + cx, v = fy y/z + cy.  K rows are (fx, fy, cx, cy).
    Broadcasts over leading dimensions.  Returns (uv, P_c)."""
    Pc = np.einsum("...ij,...j->...i", R, X) + t
    z = Pc[..., 2]
    u = K[..., 0] * Pc[..., 0] / z + K[..., 2]
    v = K[..., 1] * Pc[..., 1] / z + K[..., 3]
    return np.stack([u, v], axis=-1), Pc


def huber_rho(s: np.ndarray, delta: float) -> np.ndarray:
    """Robust loss on the squared residual norm s (Sec. 4.3 objective; the paper
    leaves rho unspecified, Huber 1964 is the reading): rho(s) = s for s <= delta^2,
    2 delta sqrt(s) - delta^2 otherwise; delta <= 0 means rho(s) = s."""
    s = np.asarray(s, dtype=np.float64)
    if delta <= 0:
        return s.copy()
    return np.where(s <= delta * delta, s, 2 * delta * np.sqrt(s) - delta * delta)


def huber_weight(s: np.ndarray, delta: float) -> np.ndarray:
    """rho'(s): 1 for s <= delta^2, delta / sqrt(s) otherwise (IRLS weight)."""
    s = np.asarray(s, dtype=np.float64)
    if delta <= 0:
        return np.ones_like(s)
    return np.where(s <= delta * delta, 1.0, delta / np.sqrt(np.maximum(s, 1e-300)))


@dataclasses.dataclass
class Problem:
    """A bundle-adjustment problem in FP64.  Poses are world->camera."""
    K: np.ndarray          # (C, 4)
    R: np.ndarray          # (C, 3, 3)
    t: np.ndarray          # (C, 3)
    X: np.ndarray          # (P, 3)
    cam: np.ndarray        # (N,)
    pt: np.ndarray         # (N,)
    uv: np.ndarray         # (N, 2)
    fixed: np.ndarray      # (C,) bool
    delta: float           # Huber delta; <= 0 plain least squares
    # prior terms (Sec. 4.3 objective); weights 0 disable them
    prior_abs: float = 0.0        # lambda_a
    prior_seq: float = 0.0        # lambda_c
    seq_k: int = 1                # sequential pairs (i, i + k), k = 1..seq_k, in camera order
    R0: np.ndarray | None = None  # T_init: the initial poses
    t0: np.ndarray | None = None
    active: np.ndarray | None = None  # (N,) bool: observations kept by the culling step
    # explicit pose-graph edges (Sec. 4.2); when given they replace the sequential pairs
    pairs: np.ndarray | None = None      # (E, 2) node indices (i, j): error T_i T_j^-1 - M_ij
    pair_meas: np.ndarray | None = None  # (E, 12) M_ij as [R | t] rows, R first
    pair_w: np.ndarray | None = None     # (E, 2) weights of the rotation and translation entries

    def __post_init__(self):
        if self.R0 is None:
            self.R0 = np.array(self.R, np.float64)
        if self.t0 is None:
            self.t0 = np.array(self.t, np.float64)
        if self.active is None:
            self.active = np.ones(self.cam.shape[0], bool)

    @classmethod
    def from_scene(cls, s, prior_abs: float = 0.0, prior_seq: float = 0.0, seq_k: int = 1) -> "Problem":
        return cls(K=np.asarray(s.K, np.float64), R=quat_to_rot(s.q0), t=np.array(s.t0, np.float64),
                   X=np.array(s.X0, np.float64), cam=np.asarray(s.obs_cam, np.int64),
                   pt=np.asarray(s.obs_pt, np.int64), uv=np.asarray(s.obs_uv, np.float64),
                   fixed=np.asarray(s.cam_fixed).astype(bool), delta=float(s.huber_delta),
                   prior_abs=float(prior_abs), prior_seq=float(prior_seq), seq_k=int(seq_k))

    @property
    def n_cams(self):
        return self.R.shape[0]

    @property
    def n_pts(self):
        return self.X.shape[0]

    @property
    def n_obs(self):
        return self.cam.shape[0]


def residuals(p: Problem, R=None, t=None, X=None):
    """Per-observation residuals r_k = pi(...) - z_k and the validity mask
    (depth > Z_MIN; masked observations get r = 0).  Observations removed by the
    culling step (``p.active`` false) also get r = 0 and count as valid: they are
    out of the problem, not masked."""
    R = p.R if R is None else R
    t = p.t if t is None else t
    X = p.X if X is None else X
    uv, Pc = project(p.K[p.cam], R[p.cam], t[p.cam], X[p.pt])
    valid = (Pc[:, 2] > Z_MIN) | ~p.active
    r = np.where((valid & p.active)[:, None], uv - p.uv, 0.0)
    return r, valid, Pc


def cost(p: Problem, R=None, t=None, X=None) -> float:
    """C = 1/2 sum_k rho(||r_k||^2) over valid observations, plus the prior terms."""
    return cost_and_masked(p, R, t, X)[0]


def cost_and_masked(p: Problem, R=None, t=None, X=None):
    """(C, number of masked observations) at a state."""
    r, valid, _ = residuals(p, R, t, X)
    s = np.sum(r * r, axis=1)
    C = 0.5 * float(np.sum(huber_rho(s, p.delta)[valid & p.active]))
    if has_priors(p):
        C += prior_cost(p, R, t)
    return C, int((~valid).sum())


# ----------------------------------------------------------------------------- prior terms

def _pose_rows(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    """The 3x4 upper part [R | t] of a pose, flattened row-major with R first:
    (R00 R01 R02 R10 ... R22, t0 t1 t2)."""
    return np.concatenate([R.reshape(-1), t])


def prior_pairs(p: Problem):
    """The relative-pose pairs: the explicit pose-graph edges when given, else the
    sequential constraint pairs (i, i + k), k = 1..seq_k, in camera order."""
    if p.pairs is not None:
        return [(int(i), int(j)) for i, j in p.pairs]
    C = p.n_cams
    return [(i, i + k) for i in range(C) for k in range(1, p.seq_k + 1) if i + k < C]


def has_priors(p: Problem) -> bool:
    return p.prior_abs > 0 or p.prior_seq > 0 or (p.pairs is not None and len(p.pairs) > 0)


def pair_row_weights(p: Problem) -> np.ndarray:
    """(n_pairs, 12) weight of each residual entry: the edge's rotation weight on the
    nine R entries and its translation weight on the three t entries; lambda_c on
    all twelve for the sequential prior."""
    n = len(prior_pairs(p))
    if p.pairs is not None:
        w = np.asarray(p.pair_w, np.float64).reshape(n, 2)
        return np.concatenate([np.repeat(w[:, :1], 9, axis=1), np.repeat(w[:, 1:], 3, axis=1)], axis=1)
    return np.full((n, 12), p.prior_seq)


def prior_residuals(p: Problem, R=None, t=None):
    """Residual 12-vectors of the prior terms: r_a,i = [R_i - R0_i | t_i - t0_i] for every
    camera (Eq. abs), and r_c,(i,j) = A - M_ij with A = T_i T_j^-1 = [R_i R_j^T | t_i - R_i R_j^T t_j]
    for every pair (Eq. seq): M_ij is the edge's measurement for explicit edges, and
    for sequential pairs A of the initial poses."""
    R = p.R if R is None else R
    t = p.t if t is None else t
    ra = np.stack([_pose_rows(R[i], t[i]) - _pose_rows(p.R0[i], p.t0[i]) for i in range(p.n_cams)])
    rc = []
    for x, (i, j) in enumerate(prior_pairs(p)):
        RA = R[i] @ R[j].T
        if p.pairs is not None:
            M = np.asarray(p.pair_meas[x], np.float64)
        else:
            RA0 = p.R0[i] @ p.R0[j].T
            M = _pose_rows(RA0, p.t0[i] - RA0 @ p.t0[j])
        rc.append(_pose_rows(RA, t[i] - RA @ t[j]) - M)
    return ra, np.array(rc).reshape(-1, 12)


def prior_cost(p: Problem, R=None, t=None) -> float:
    """1/2 (lambda_a sum_i ||r_a,i||^2 + sum_pairs sum_q w_q r_c,q^2)."""
    ra, rc = prior_residuals(p, R, t)
    return 0.5 * (p.prior_abs * float(np.sum(ra * ra)) + float(np.sum(pair_row_weights(p) * rc * rc)))


def _rows_of_left_increment(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    """d[R | t]/d xi for T <- Exp(xi) T, xi = (rho, phi): the rotation rows change by
    [e_m]x R for phi_m, the translation rows by rho and by [phi]x t = -[t]x phi.
    Returns the 12 x 6 Jacobian in the _pose_rows order."""
    J = np.zeros((12, 6))
    for m in range(3):
        e = np.zeros(3)
        e[m] = 1.0
        J[:9, 3 + m] = (hat(e) @ R).reshape(-1)
    J[9:, :3] = np.eye(3)
    J[9:, 3:] = -hat(t)
    return J


def prior_jacobians(p: Problem, R=None, t=None):
    """Jacobians of the prior residuals for left increments of the poses.
    Absolute term of camera i: _rows_of_left_increment(R_i, t_i).  Sequential term of
    (i, j): A <- Exp(xi_i) A Exp(-xi_j), so d/dxi_i = _rows_of_left_increment(R_A, t_A)
    and d/dxi_j has rotation rows -R_A [e_m]x (phi_m) and translation rows -R_A (rho).
    Returns (Ja (C, 12, 6), Jci (n, 12, 6), Jcj (n, 12, 6))."""
    R = p.R if R is None else R
    t = p.t if t is None else t
    Ja = np.stack([_rows_of_left_increment(R[i], t[i]) for i in range(p.n_cams)])
    Jci, Jcj = [], []
    for i, j in prior_pairs(p):
        RA = R[i] @ R[j].T
        tA = t[i] - RA @ t[j]
        Jci.append(_rows_of_left_increment(RA, tA))
        Jj = np.zeros((12, 6))
        for m in range(3):
            e = np.zeros(3)
            e[m] = 1.0
            Jj[:9, 3 + m] = (-RA @ hat(e)).reshape(-1)
        Jj[9:, :3] = -RA
        Jcj.append(Jj)
    return Ja, np.array(Jci).reshape(-1, 12, 6), np.array(Jcj).reshape(-1, 12, 6)


def prior_system(p: Problem, n: int):
    """Rows of the weighted prior residuals over the unknowns [free camera increments |
    point increments] (n columns): sqrt(lambda) J and sqrt(lambda) r, so that they add
    J^T J to H and J^T r to g.  Fixed cameras contribute no columns."""
    fidx, _ = _free_index(p.fixed)
    ra, rc = prior_residuals(p)
    Ja, Jci, Jcj = prior_jacobians(p)
    rows, cols, vals, rhs = [], [], [], []
    row = 0
    sa = math.sqrt(p.prior_abs)
    sw = np.sqrt(pair_row_weights(p))
    if p.prior_abs > 0:
        for i in range(p.n_cams):
            if fidx[i] >= 0:
                for q in range(12):
                    for m in range(6):
                        rows.append(row + q)
                        cols.append(6 * fidx[i] + m)
                        vals.append(sa * Ja[i, q, m])
                rhs.append(sa * ra[i])
                row += 12
    for x, (i, j) in enumerate(prior_pairs(p)):
        if fidx[i] < 0 and fidx[j] < 0:
            continue
        for cam, Jx in ((i, Jci[x]), (j, Jcj[x])):
            if fidx[cam] >= 0:
                for q in range(12):
                    for m in range(6):
                        rows.append(row + q)
                        cols.append(6 * fidx[cam] + m)
                        vals.append(sw[x, q] * Jx[q, m])
        rhs.append(sw[x] * rc[x])
        row += 12
    Jp = sp.csr_matrix((np.array(vals), (np.array(rows, np.int64), np.array(cols, np.int64))), shape=(row, n))
    return Jp, (np.concatenate(rhs) if rhs else np.zeros(0))


def rms(p: Problem, R=None, t=None, X=None, inlier_px: float | None = None) -> float:
    """sqrt(sum ||r||^2 / N) in pixels over valid active observations (unweighted);
    with ``inlier_px``, over observations with ||r|| <= inlier_px only."""
    r, valid, _ = residuals(p, R, t, X)
    s = np.sum(r * r, axis=1)
    m = valid & p.active
    if inlier_px is not None:
        m = m & (s <= inlier_px * inlier_px)
    return math.sqrt(float(np.sum(s[m])) / max(int(m.sum()), 1))


def jacobians(p: Problem, R=None, t=None, X=None):
    """Analytic Jacobians of r_k for a left increment T <- Exp(xi) T (xi = (rho, phi))
    and an additive point increment:
      J_pi = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]],
      J_c  = J_pi [I | -[P_c]x]   (2 x 6),
      J_p  = J_pi R               (2 x 3).
    Masked observations get zero rows."""
    R = p.R if R is None else R
    t = p.t if t is None else t
    X = p.X if X is None else X
    _, valid, Pc = residuals(p, R, t, X)
    Kk = p.K[p.cam]
    x, y, z = Pc[:, 0], Pc[:, 1], Pc[:, 2]
    zs = np.where(valid & (z > Z_MIN), z, 1.0)
    Jpi = np.zeros((p.n_obs, 2, 3))
    Jpi[:, 0, 0] = Kk[:, 0] / zs
    Jpi[:, 0, 2] = -Kk[:, 0] * x / (zs * zs)
    Jpi[:, 1, 1] = Kk[:, 1] / zs
    Jpi[:, 1, 2] = -Kk[:, 1] * y / (zs * zs)
    Jpi[~(valid & p.active)] = 0.0
    dP = np.concatenate([np.broadcast_to(np.eye(3), (p.n_obs, 3, 3)), -hat(Pc)], axis=2)
    Jc = Jpi @ dP
    Jp = Jpi @ R[p.cam]
    return Jc, Jp


# ----------------------------------------------------------------------------- parameter layout

def _free_index(fixed: np.ndarray):
    idx = -np.ones(fixed.size, np.int64)
    free = np.nonzero(~fixed)[0]
    idx[free] = np.arange(free.size)
    return idx, free.size


def apply_step(p: Problem, dc: np.ndarray, dp: np.ndarray):
    """Trial state: T_i <- Exp(dc_i) T_i for free cameras, X_j <- X_j + dp_j."""
    fidx, nf = _free_index(p.fixed)
    R = p.R.copy()
    t = p.t.copy()
    free = np.nonzero(~p.fixed)[0]
    if nf:
        dR, dt = se3_exp(dc.reshape(nf, 6))
        R[free] = dR @ p.R[free]
        t[free] = np.einsum("nij,nj->ni", dR, p.t[free]) + dt
    X = p.X + dp.reshape(-1, 3)
    return R, t, X


def normal_equations(p: Problem):
    """Full Gauss-Newton system over [free camera increments | point increments]:
    H = sum_k w_k J_k^T J_k, g = sum_k w_k J_k^T r_k with w_k = rho'(||r_k||^2),
    built from the sparse 2N x n Jacobian.  Returns (H sparse CSR, g, J, w, r)."""
    r, valid, _ = residuals(p)
    Jc, Jp = jacobians(p)
    s = np.sum(r * r, axis=1)
    w = np.where(valid & p.active, huber_weight(s, p.delta), 0.0)
    fidx, nf = _free_index(p.fixed)
    N = p.n_obs
    ncam = 6 * nf
    n = ncam + 3 * p.n_pts
    rows, cols, vals = [], [], []
    ci = fidx[p.cam]
    has_c = ci >= 0
    for comp in range(2):
        rr = 2 * np.arange(N) + comp
        for m in range(6):
            rows.append(rr[has_c])
            cols.append(6 * ci[has_c] + m)
            vals.append(Jc[has_c, comp, m])
        for m in range(3):
            rows.append(rr)
            cols.append(ncam + 3 * p.pt + m)
            vals.append(Jp[:, comp, m])
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * N, n))
    Wd = sp.diags(np.repeat(w, 2))
    H = (J.T @ Wd @ J).tocsr()
    g = J.T @ (np.repeat(w, 2) * r.reshape(-1))
    if has_priors(p):
        Jp, rp = prior_system(p, n)
        H = (H + Jp.T @ Jp).tocsr()
        g = g + Jp.T @ rp
    return H, np.asarray(g).ravel(), J, w, r


def damping_diag(Hdiag: np.ndarray) -> np.ndarray:
    """Marquardt scaling D = diag(H) clamped to [1e-6, 1e32]."""
    return np.clip(Hdiag, D_MIN, D_MAX)


# ----------------------------------------------------------------------------- LM driver

@dataclasses.dataclass
class LMOptions:
    max_iters: int = 20
    lambda0: float = 1e-4
    solve: str = "exact"        # lm_schur: "exact" or "pcg"
    pcg_max_iters: int = 50
    pcg_rel_tol: float = 1e-6


@dataclasses.dataclass
class LMResult:
    R: np.ndarray
    t: np.ndarray
    X: np.ndarray
    iter_cost: list            # C_0, C_1, ..., C_n (accepted-state cost after each iteration)
    lambdas: list              # lambda used for the step of each iteration
    accepted: list             # bool per iteration
    rhos: list
    pcg_iters: list
    status: int
    nus: list = dataclasses.field(default_factory=list)   # nu after each iteration


def lm_iterate(state, opts: LMOptions, cost_fn, linearize, solve, apply):
    """The Levenberg-Marquardt iteration (Madsen, Nielsen, Tingleff 2004, Sec. 3.2,
    with Marquardt's diagonal scaling), independent of what the unknowns are.

    ``cost_fn(state) -> (C, masked)``, ``linearize(state) -> (H, g)`` of the model
    C(x + d) ~ C + g^T d + d^T H d / 2, ``solve(state, H, g, D, lam) -> (d, pcg_its)``
    for (H + lam diag(D)) d = -g (d None if the damped system is not numerically
    positive definite) and ``apply(state, d) -> trial state``.

    One iteration = one linearisation (kept after a rejected step), one damped solve
    and one trial cost.  D = diag(H) clamped to [1e-6, 1e32].  The predicted decrease
    of the undamped model is dL = -g^T d - d^T H d / 2 = d^T (lam D d - g) / 2, the gain
    ratio rho = (C - C_trial) / dL.  The step is accepted iff rho > 1e-3, dL > 0, the
    trial cost is finite and the trial state masks no more observations (depth <= Z_MIN)
    than the current one -- a step may not lower the cost by pushing points behind
    their cameras.  On accept lam *= max(1/3, 1 - (2 rho - 1)^3) and nu = 2; on reject
    (including a failed solve) lam *= nu and nu *= 2.  lam is clamped to
    [1e-12, 1e16].  The count is fixed (no early stop); a run that ends with lam at its
    upper clamp reports STATUS_DAMPING, a non-finite final cost STATUS_NUMERICAL.
    Returns (final state, LMResult without R, t, X)."""
    lam = opts.lambda0
    nu = 2.0
    C, masked = cost_fn(state)
    out = LMResult(None, None, None, [C], [], [], [], [], STATUS_OK)
    lin = None
    for _ in range(opts.max_iters):
        if lin is None:
            lin = linearize(state)
        H, g = lin
        D = damping_diag(H.diagonal())
        delta, pcg_it = solve(state, H, g, D, lam)
        out.lambdas.append(lam)
        out.pcg_iters.append(pcg_it)
        accept = False
        if delta is None:
            rho = float("nan")
        else:
            dL = 0.5 * float(delta @ (lam * D * delta - g))
            trial = apply(state, delta)
            Cn, masked_n = cost_fn(trial)
            rho = (C - Cn) / dL if dL != 0 else -np.inf
            accept = bool(np.isfinite(Cn) and dL > 0 and rho > ACCEPT_RHO and masked_n <= masked)
        out.rhos.append(rho)
        if accept:
            state, C, masked = trial, Cn, masked_n
            lam = lam * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
            lin = None
        else:
            lam = lam * nu
            nu = 2.0 * nu
        lam = min(max(lam, LAMBDA_MIN), LAMBDA_MAX)
        out.accepted.append(accept)
        out.nus.append(nu)
        out.iter_cost.append(C)
    if not np.isfinite(C):
        out.status = STATUS_NUMERICAL
    elif lam >= LAMBDA_MAX:
        out.status = STATUS_DAMPING
    return state, out


def _lm_loop(p: Problem, opts: LMOptions, solve_step):
    """LM over the cameras and points of a BA problem (``lm_iterate``), the state
    being the problem itself; ``solve_step(p, H, g, D, lam, opts)`` solves the damped
    normal equations for d = (d_cameras, d_points)."""
    p = dataclasses.replace(p, R=p.R.copy(), t=p.t.copy(), X=p.X.copy())
    nf = int((~p.fixed).sum())

    def linearize(q):
        H, g = normal_equations(q)[:2]
        return H, g

    def apply(q, delta):
        Rn, tn, Xn = apply_step(q, delta[:6 * nf], delta[6 * nf:])
        return dataclasses.replace(q, R=Rn, t=tn, X=Xn)

    p, out = lm_iterate(p, opts, cost_and_masked, linearize,
                        lambda q, H, g, D, lam: solve_step(q, H, g, D, lam, opts), apply)
    out.R, out.t, out.X = p.R, p.t, p.X
    return out


def _dense_step(p, H, g, D, lam, opts):
    A = H.toarray()
    A[np.diag_indices_from(A)] += lam * D
    try:
        c = scipy.linalg.cho_factor(A, lower=True)
    except np.linalg.LinAlgError:
        return None, 0
    return scipy.linalg.cho_solve(c, -g), 0


def lm_dense(p: Problem, opts: LMOptions | None = None) -> LMResult:
    """O1: LM with the full damped normal equations solved by dense Cholesky."""
    return _lm_loop(p, opts or LMOptions(), _dense_step)


# ----------------------------------------------------------------------------- Schur complement

def schur_blocks(H: sp.csr_matrix, g: np.ndarray, D: np.ndarray, lam: float, ncam: int):
    """Split the damped system [[U*, W], [W^T, V*]] [dc; dp] = [-g_c; -g_p] and form
    the reduced camera system S dc = b with S = U* - W V*^-1 W^T and
    b = -g_c + W V*^-1 g_p (Triggs et al. 2000, Sec. 6.1).  V* is block diagonal
    with 3x3 blocks, inverted block by block.  Returns (S dense, b, Vinv sparse, W)."""
    Hd = H.tocsr()
    n = Hd.shape[0]
    damp = sp.diags(lam * D)
    A = (Hd + damp).tocsr()
    U = A[:ncam, :ncam].toarray()
    W = A[:ncam, ncam:].tocsr()
    V = A[ncam:, ncam:].tocsr()
    npts = (n - ncam) // 3
    Vb = np.zeros((npts, 3, 3))
    Vcoo = V.tocoo()
    Vb[Vcoo.row // 3, Vcoo.row % 3, Vcoo.col % 3] = Vcoo.data
    Vinv_b = np.linalg.inv(Vb)
    ii = np.repeat(np.arange(npts), 9) * 3 + np.tile(np.repeat(np.arange(3), 3), npts)
    jj = np.repeat(np.arange(npts), 9) * 3 + np.tile(np.arange(3), 3 * npts)
    Vinv = sp.csr_matrix((Vinv_b.reshape(-1), (ii, jj)), shape=(3 * npts, 3 * npts))
    Y = (W @ Vinv).tocsr()
    S = U - (Y @ W.T).toarray()
    gc, gp = g[:ncam], g[ncam:]
    b = -gc + Y @ gp
    return S, np.asarray(b).ravel(), Vinv, W


def pcg_block_jacobi(S: np.ndarray, b: np.ndarray, tol: float, max_iters: int):
    """Preconditioned CG (Hestenes-Stiefel 1952) on S x = b with the block-Jacobi
    preconditioner M = blockdiag(S_aa) of 6x6 camera blocks.  x0 = 0.  Stops when
    ||r||_2 <= tol ||b||_2 (unpreconditioned residual) or after ``max_iters``
    products with S, or if p^T S p <= 0.  Returns (x, iterations)."""
    n = b.size
    nb = n // 6
    Minv = np.zeros((nb, 6, 6))
    for a in range(nb):
        blk = S[6 * a:6 * a + 6, 6 * a:6 * a + 6]
        L = np.linalg.cholesky(blk)
        Li = np.linalg.inv(L)
        Minv[a] = Li.T @ Li

    def prec(r):
        return np.einsum("aij,aj->ai", Minv, r.reshape(nb, 6)).reshape(-1)

    x = np.zeros(n)
    r = b.copy()
    bn = math.sqrt(float(b @ b))
    if bn == 0.0:
        return x, 0
    z = prec(r)
    pdir = z.copy()
    rz = float(r @ z)
    it = 0
    while it < max_iters:
        q = S @ pdir
        pq = float(pdir @ q)
        it += 1
        if not pq > 0:
            break
        alpha = rz / pq
        x = x + alpha * pdir
        r = r - alpha * q
        if math.sqrt(float(r @ r)) <= tol * bn:
            break
        z = prec(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        pdir = z + beta * pdir
        rz = rz_new
    return x, it


def _schur_step(p, H, g, D, lam, opts):
    nf = int((~p.fixed).sum())
    ncam = 6 * nf
    S, b, Vinv, W = schur_blocks(H, g, D, lam, ncam)
    if opts.solve == "exact":
        try:
            c = scipy.linalg.cho_factor(S, lower=True)
        except np.linalg.LinAlgError:
            return None, 0
        dc = scipy.linalg.cho_solve(c, b)
        it = 0
    else:
        dc, it = pcg_block_jacobi(S, b, opts.pcg_rel_tol, opts.pcg_max_iters)
    gp = g[ncam:]
    dp = Vinv @ (-gp - W.T @ dc)
    return np.concatenate([dc, np.asarray(dp).ravel()]), it


def lm_schur(p: Problem, opts: LMOptions | None = None) -> LMResult:
    """O2: LM with points eliminated (explicit Schur complement), the reduced
    camera system solved exactly (dense Cholesky) or by block-Jacobi PCG."""
    return _lm_loop(p, opts or LMOptions(solve="exact"), _schur_step)


# ----------------------------------------------------------------------------- pose-only GN

def pose_only_gn(K, q0, t0, X, uv, delta: float, iters: int = 10):
    """Gauss-Newton on one world->camera pose with the map points fixed (the
    localization mode of Sec. 6.4.2).  Each iteration: IRLS weights w = rho'(s),
    H = sum w J_c^T J_c, g = sum w J_c^T r, delta = -H^-1 g by Cholesky, T <- Exp(delta) T.
    No damping and no rejection; if H is not positive definite the update is skipped
    and the status flag set.  Returns (R, t, status, costs)."""
    R = quat_to_rot(np.asarray(q0, np.float64))
    t = np.array(t0, np.float64)
    X = np.asarray(X, np.float64)
    uv = np.asarray(uv, np.float64)
    K = np.asarray(K, np.float64)
    status = 0
    costs = []
    for _ in range(iters):
        pr, Pc = project(K[None, :], R[None], t[None], X)
        valid = Pc[:, 2] > Z_MIN
        r = np.where(valid[:, None], pr - uv, 0.0)
        s = np.sum(r * r, axis=1)
        w = np.where(valid, huber_weight(s, delta), 0.0)
        costs.append(0.5 * float(np.sum(huber_rho(s, delta)[valid])))
        x, y, z = Pc[:, 0], Pc[:, 1], np.where(valid, Pc[:, 2], 1.0)
        Jpi = np.zeros((X.shape[0], 2, 3))
        Jpi[:, 0, 0] = K[0] / z
        Jpi[:, 0, 2] = -K[0] * x / (z * z)
        Jpi[:, 1, 1] = K[1] / z
        Jpi[:, 1, 2] = -K[1] * y / (z * z)
        dP = np.concatenate([np.broadcast_to(np.eye(3), (X.shape[0], 3, 3)), -hat(Pc)], axis=2)
        Jc = Jpi @ dP
        H = np.einsum("n,nki,nkj->ij", w, Jc, Jc)
        g = np.einsum("n,nki,nk->i", w, Jc, r)
        try:
            L = np.linalg.cholesky(H)
        except np.linalg.LinAlgError:
            status = 1
            continue
        d = -scipy.linalg.cho_solve((L, True), g)
        dR, dt = se3_exp(d)
        R = dR @ R
        t = dR @ t + dt
    pr, Pc = project(K[None, :], R[None], t[None], X)
    valid = Pc[:, 2] > Z_MIN
    r = np.where(valid[:, None], pr - uv, 0.0)
    costs.append(0.5 * float(np.sum(huber_rho(np.sum(r * r, axis=1), delta)[valid])))
    return R, t, status, costs


# ----------------------------------------------------------------------------- triangulation and culling

def triangulate_midpoint(p: Problem, j: int, R=None, t=None):
    """Multi-view midpoint triangulation of point j from its active observations
    (Sec. 4.3 names the DLT of Eq. dlt and a midpoint method; this is the latter):
    X = argmin sum_k ||(I - d_k d_k^T)(X - c_k)||^2 with camera centre c_k = -R_k^T t_k and
    unit ray d_k along R_k^T K_k^-1 (u, v, 1), i.e. the solution of
    (sum_k (I - d_k d_k^T)) X = sum_k (I - d_k d_k^T) c_k (numpy.linalg.solve).
    Returns (X, ok): ok iff at least two active observations, det of the 3x3 system
    > 1e-12 and every active observation has depth > Z_MIN at X."""
    R = p.R if R is None else R
    t = p.t if t is None else t
    ks = np.nonzero((p.pt == j) & p.active)[0]
    if ks.size < 2:
        return None, False
    A = np.zeros((3, 3))
    b = np.zeros(3)
    for k in ks:
        i = p.cam[k]
        fx, fy, cx, cy = p.K[i]
        d = R[i].T @ np.array([(p.uv[k, 0] - cx) / fx, (p.uv[k, 1] - cy) / fy, 1.0])
        d = d / np.linalg.norm(d)
        c = -R[i].T @ t[i]
        M = np.eye(3) - np.outer(d, d)
        A += M
        b += M @ c
    if not np.linalg.det(A) > 1e-12:
        return None, False
    X = np.linalg.solve(A, b)
    for k in ks:
        i = p.cam[k]
        if not (R[i][2] @ X + t[i][2]) > Z_MIN:
            return None, False
    return X, True


def cull_and_triangulate(p: Problem, tau_px: float, method: str = "midpoint"):
    """The culling step after a BA round (Sec. 4.3): an active observation stays
    active iff ||r_k|| <= tau_px at the current state; a point left with fewer than two
    active observations leaves the problem (all its observations inactive); a point
    that lost observations is re-triangulated from the ones that remain (midpoint, or
    DLT with method="dlt"), and leaves the problem if that fails.  Updates p.active and p.X in place and
    returns (active observations, points in the problem)."""
    r, valid, _ = residuals(p)
    s = np.sum(r * r, axis=1)
    keep = p.active & valid & (s <= tau_px * tau_px)
    lost = p.active & ~keep
    p.active = keep
    tri = triangulate_midpoint if method == "midpoint" else triangulate_dlt
    for j in np.unique(p.pt[lost]):
        n = int(np.count_nonzero((p.pt == j) & p.active))
        X, ok = tri(p, j) if n >= 2 else (None, False)
        if ok:
            p.X[j] = X
        else:
            p.active[p.pt == j] = False
    counts = np.bincount(p.pt[p.active], minlength=p.n_pts)
    return int(p.active.sum()), int(np.count_nonzero(counts > 0))


def refine(p: Problem, stages, rounds: int, opts: LMOptions):
    """The two-stage iterative framework of Sec. 4.3: for each stage (huber_delta,
    tau_px[, method]) -- first a robust loss with a relaxed threshold, then no loss with a
    strict one -- ``rounds`` times: an LM solve from lambda0, then cull_and_triangulate.
    Returns (p, history) with one (stage, round, cost, active obs, points) per round."""
    p = dataclasses.replace(p, R=p.R.copy(), t=p.t.copy(), X=p.X.copy(), active=p.active.copy())
    hist = []
    for si, stage in enumerate(stages):
        delta, tau = stage[0], stage[1]
        method = stage[2] if len(stage) > 2 else "midpoint"
        p.delta = float(delta)
        for rd in range(rounds):
            res = lm_schur(p, opts)
            p.R, p.t, p.X = res.R, res.t, res.X
            n_act, n_pts = cull_and_triangulate(p, tau, method)
            hist.append((si, rd, res.iter_cost[-1], n_act, n_pts))
    return p, hist


# ----------------------------------------------------------------------------- pose graph

def pose_graph_problem(R0, t0, fixed, edges, meas_R, meas_t, w_rot, w_trans, prior_abs: float = 0.0):
    """A pose graph (Sec. 4.2) as a Problem with no observations: nodes with initial
    world->camera poses (R0, t0), hard-fixed nodes, and edges (i, j) with measured
    relative poses M_ij = (meas_R, meas_t) of A_ij = T_i T_j^-1 and per-edge weights of
    the rotation and translation entries, so that
    C = 1/2 sum_e (w_rot ||R_A - R_M||_F^2 + w_trans ||t_A - t_M||^2)
        + 1/2 prior_abs sum_i ||T_i - T_i,init||^2.
    Sequential, loop-closure and extrinsic edges differ only in where M comes from."""
    R0 = np.asarray(R0, np.float64)
    C = R0.shape[0]
    edges = np.asarray(edges, np.int64).reshape(-1, 2)
    meas = np.concatenate([np.asarray(meas_R, np.float64).reshape(-1, 9),
                           np.asarray(meas_t, np.float64).reshape(-1, 3)], axis=1)
    w = np.stack([np.broadcast_to(np.asarray(w_rot, np.float64), edges.shape[0]),
                  np.broadcast_to(np.asarray(w_trans, np.float64), edges.shape[0])], axis=1)
    return Problem(K=np.ones((C, 4)), R=R0.copy(), t=np.array(t0, np.float64), X=np.zeros((0, 3)),
                   cam=np.zeros(0, np.int64), pt=np.zeros(0, np.int64), uv=np.zeros((0, 2)),
                   fixed=np.asarray(fixed).astype(bool), delta=0.0, prior_abs=float(prior_abs),
                   pairs=edges, pair_meas=meas, pair_w=w)


# ----------------------------------------------------------------------------- vehicle-rig BA

@dataclasses.dataclass
class RigProblem:
    """Bundle adjustment in the vehicle-rig configuration (Sec. 4.4): the pose of rig
    camera c at frame f is the composition T_(f,c) = E_c T_v(f) of the camera's extrinsic
    E_c = T_c^v (vehicle -> camera) and the vehicle pose T_v(f) (world -> vehicle), both
    unknown; extrinsics are shared by every frame.  Terms: the reprojection error of
    Sec. 4.4 (with rho and the masking of the BA problem), the absolute prior on the
    extrinsics 1/2 lambda_e sum_c ||E_c - E_c,init||^2 and the rigidity constraints
    of Eq. extrinsic between rig cameras, which in this configuration depend on the
    extrinsics alone: 1/2 lambda_r ||E_c E_d^-1 - E_c,init E_d,init^-1||^2."""
    K: np.ndarray          # (nr, 4) intrinsics of each rig camera
    Rv: np.ndarray         # (F, 3, 3) world -> vehicle
    tv: np.ndarray         # (F, 3)
    Re: np.ndarray         # (nr, 3, 3) vehicle -> camera
    te: np.ndarray         # (nr, 3)
    X: np.ndarray          # (P, 3)
    frame: np.ndarray      # (N,)
    rcam: np.ndarray       # (N,)
    pt: np.ndarray         # (N,)
    uv: np.ndarray         # (N, 2)
    fixed_v: np.ndarray    # (F,) bool
    fixed_e: np.ndarray    # (nr,) bool
    delta: float
    prior_ext: float = 0.0             # lambda_e
    rig_pairs: np.ndarray | None = None  # (E, 2) rig camera pairs of the rigidity terms
    prior_rig: float = 0.0             # lambda_r
    Re0: np.ndarray | None = None
    te0: np.ndarray | None = None

    def __post_init__(self):
        if self.Re0 is None:
            self.Re0 = np.array(self.Re, np.float64)
        if self.te0 is None:
            self.te0 = np.array(self.te, np.float64)
        if self.rig_pairs is None:
            self.rig_pairs = np.zeros((0, 2), np.int64)

    @property
    def n_frames(self):
        return self.Rv.shape[0]

    @property
    def n_rig(self):
        return self.Re.shape[0]


def rig_adjoint(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Ad_E for E = (R, t) acting on xi = (rho, phi): E Exp(xi) E^-1 = Exp(Ad_E xi),
    Ad_E = [[R, [t]x R], [0, R]]."""
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[:3, 3:] = hat(t) @ R
    A[3:, 3:] = R
    return A


def rig_camera_problem(q: RigProblem, Rv=None, tv=None, Re=None, te=None, X=None) -> Problem:
    """The same observations as a BA problem over the composed cameras (f, c), camera
    index f * nr + c, T_(f,c) = E_c T_v(f): R = R_e R_v, t = R_e t_v + t_e."""
    Rv = q.Rv if Rv is None else Rv
    tv = q.tv if tv is None else tv
    Re = q.Re if Re is None else Re
    te = q.te if te is None else te
    X = q.X if X is None else X
    F, nr = Rv.shape[0], Re.shape[0]
    R = np.einsum("cij,fjk->fcik", Re, Rv).reshape(F * nr, 3, 3)
    t = (np.einsum("cij,fj->fci", Re, tv) + te[None]).reshape(F * nr, 3)
    return Problem(K=np.tile(q.K, (F, 1)), R=R, t=t, X=X, cam=q.frame * nr + q.rcam, pt=q.pt, uv=q.uv,
                   fixed=np.zeros(F * nr, bool), delta=q.delta)


def rig_extrinsic_view(q: RigProblem, Re=None, te=None) -> Problem:
    """The extrinsic terms as relative-pose priors over the extrinsics: the absolute
    prior (lambda_e, anchored at the initial extrinsics) and the rigidity pairs (weight
    lambda_r on every entry, measured from the initial extrinsics)."""
    Re = q.Re if Re is None else Re
    te = q.te if te is None else te
    nr = Re.shape[0]
    meas = []
    for c, d in q.rig_pairs:
        RA = q.Re0[c] @ q.Re0[d].T
        meas.append(_pose_rows(RA, q.te0[c] - RA @ q.te0[d]))
    return Problem(K=np.ones((nr, 4)), R=Re, t=te, X=np.zeros((0, 3)), cam=np.zeros(0, np.int64),
                   pt=np.zeros(0, np.int64), uv=np.zeros((0, 2)), fixed=np.asarray(q.fixed_e, bool), delta=0.0,
                   prior_abs=q.prior_ext, R0=q.Re0, t0=q.te0, pairs=np.asarray(q.rig_pairs, np.int64).reshape(-1, 2),
                   pair_meas=np.array(meas).reshape(-1, 12),
                   pair_w=np.full((len(q.rig_pairs), 2), q.prior_rig))


def rig_cost_and_masked(q: RigProblem, Rv=None, tv=None, Re=None, te=None, X=None):
    C, masked = cost_and_masked(rig_camera_problem(q, Rv, tv, Re, te, X))
    v = rig_extrinsic_view(q, Re, te)
    if has_priors(v):
        C += prior_cost(v)
    return C, masked


def rig_normal_equations(q: RigProblem):
    """H = J^T W J and g = J^T W r over [free vehicle increments | free extrinsic
    increments | point increments], with the camera Jacobian of each observation split
    by the chain rule: d/dxi_v = J_c Ad_(E_c) (T_v <- Exp(xi_v) T_v moves the camera by
    Exp(Ad_E xi_v)), d/dxi_e = J_c; plus the extrinsic prior rows."""
    p = rig_camera_problem(q)
    r, valid, _ = residuals(p)
    Jc, Jp = jacobians(p)
    s = np.sum(r * r, axis=1)
    w = np.where(valid & p.active, huber_weight(s, p.delta), 0.0)
    vidx, nv = _free_index(np.asarray(q.fixed_v, bool))
    eidx, ne = _free_index(np.asarray(q.fixed_e, bool))
    N = p.n_obs
    n = 6 * nv + 6 * ne + 3 * q.X.shape[0]
    Ad = np.stack([rig_adjoint(q.Re[c], q.te[c]) for c in range(q.n_rig)])
    Jv = np.einsum("nij,njk->nik", Jc, Ad[q.rcam])
    rows, cols, vals = [], [], []
    fv, fe = vidx[q.frame], eidx[q.rcam]
    for comp in range(2):
        rr = 2 * np.arange(N) + comp
        for m in range(6):
            hv, he = fv >= 0, fe >= 0
            rows += [rr[hv], rr[he]]
            cols += [6 * fv[hv] + m, 6 * nv + 6 * fe[he] + m]
            vals += [Jv[hv, comp, m], Jc[he, comp, m]]
        for m in range(3):
            rows.append(rr)
            cols.append(6 * nv + 6 * ne + 3 * q.pt + m)
            vals.append(Jp[:, comp, m])
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(2 * N, n))
    Wd = sp.diags(np.repeat(w, 2))
    H = (J.T @ Wd @ J).tocsr()
    g = J.T @ (np.repeat(w, 2) * r.reshape(-1))
    v = rig_extrinsic_view(q)
    if has_priors(v):
        Jr, rp = prior_system(v, 6 * ne)
        Jr = sp.hstack([sp.csr_matrix((Jr.shape[0], 6 * nv)), Jr, sp.csr_matrix((Jr.shape[0], 3 * q.X.shape[0]))])
        H = (H + Jr.T @ Jr).tocsr()
        g = g + Jr.T @ rp
    return H, np.asarray(g).ravel()


def rig_apply_step(q: RigProblem, delta: np.ndarray):
    """T_v(f) <- Exp(d_v) T_v(f), E_c <- Exp(d_e) E_c for free ones, X <- X + d_p."""
    vidx, nv = _free_index(np.asarray(q.fixed_v, bool))
    eidx, ne = _free_index(np.asarray(q.fixed_e, bool))
    Rv, tv, Re, te = q.Rv.copy(), q.tv.copy(), q.Re.copy(), q.te.copy()
    fv, fe = np.nonzero(vidx >= 0)[0], np.nonzero(eidx >= 0)[0]
    if nv:
        dR, dt = se3_exp(delta[:6 * nv].reshape(nv, 6))
        Rv[fv] = dR @ q.Rv[fv]
        tv[fv] = np.einsum("nij,nj->ni", dR, q.tv[fv]) + dt
    if ne:
        dR, dt = se3_exp(delta[6 * nv:6 * (nv + ne)].reshape(ne, 6))
        Re[fe] = dR @ q.Re[fe]
        te[fe] = np.einsum("nij,nj->ni", dR, q.te[fe]) + dt
    X = q.X + delta[6 * (nv + ne):].reshape(-1, 3)
    return Rv, tv, Re, te, X


def lm_rig(q: RigProblem, opts: LMOptions | None = None) -> LMResult:
    """Levenberg-Marquardt (``lm_iterate``) on the vehicle-rig problem: Marquardt
    scaling on the rig Hessian's diagonal, the damped normal equations solved by dense
    Cholesky.  The result's R, t hold the vehicle poses; the extrinsics are returned in
    ``ext`` = (Re, te)."""
    opts = opts or LMOptions()
    q = dataclasses.replace(q, Rv=q.Rv.copy(), tv=q.tv.copy(), Re=q.Re.copy(), te=q.te.copy(), X=q.X.copy())

    def apply(r, delta):
        Rv, tv, Re, te, X = rig_apply_step(r, delta)
        return dataclasses.replace(r, Rv=Rv, tv=tv, Re=Re, te=te, X=X)

    q, out = lm_iterate(q, opts, rig_cost_and_masked, rig_normal_equations,
                        lambda r, H, g, D, lam: _dense_step(None, H, g, D, lam, opts), apply)
    out.R, out.t, out.X = q.Rv, q.tv, q.X
    out.ext = (q.Re, q.te)
    return out


def triangulate_dlt(p: Problem, j: int, R=None, t=None):
    """DLT triangulation of point j from its active observations (Eq. dlt), read as the
    classical homogeneous linear method in normalized camera coordinates: with
    (x, y) = K^-1 (u, v) and P = [R | t], each observation gives the rows x P_3 - P_1 and
    y P_3 - P_2 of A, which express p x (P X~) = 0; X~ minimises ||A X~|| over
    ||X~|| = 1, the right singular vector of A for its smallest singular value
    (numpy.linalg.svd), and X = X~[:3] / X~[3].  Returns (X, ok): ok iff at least two
    active observations, |X~[3]| > 1e-12 and every active observation has depth > Z_MIN."""
    R = p.R if R is None else R
    t = p.t if t is None else t
    ks = np.nonzero((p.pt == j) & p.active)[0]
    if ks.size < 2:
        return None, False
    rows = []
    for k in ks:
        i = p.cam[k]
        fx, fy, cx, cy = p.K[i]
        x, y = (p.uv[k, 0] - cx) / fx, (p.uv[k, 1] - cy) / fy
        P = np.concatenate([R[i], t[i][:, None]], axis=1)
        rows.append(x * P[2] - P[0])
        rows.append(y * P[2] - P[1])
    _, _, Vt = np.linalg.svd(np.array(rows))
    Xh = Vt[-1]
    if not abs(Xh[3]) > 1e-12:
        return None, False
    X = Xh[:3] / Xh[3]
    for k in ks:
        i = p.cam[k]
        if not (R[i][2] @ X + t[i][2]) > Z_MIN:
            return None, False
    return X, True


def triangulate_points(p: Problem, method: str = "midpoint"):
    """Every point triangulated from scratch from its active observations, by the midpoint
    or the DLT method.  Returns (X (P, 3), ok (P,) bool); X is the input point where
    ok is false."""
    f = triangulate_midpoint if method == "midpoint" else triangulate_dlt
    X = np.array(p.X, np.float64)
    ok = np.zeros(p.n_pts, bool)
    for j in range(p.n_pts):
        Xj, okj = f(p, j)
        if okj:
            X[j], ok[j] = Xj, True
    return X, ok


def ransac_pair(h: int, n: int):
    """Observation pair of hypothesis h on a track of n observations (a fixed schedule
    that lists every ordered pair once within its first n (n - 1) hypotheses):
    a = h mod n, b = (a + 1 + (h div n) mod (n - 1)) mod n."""
    a = h % n
    return a, (a + 1 + (h // n) % (n - 1)) % n


def triangulate_ransac(p: Problem, j: int, tau_px: float, n_hyp: int, method: str = "midpoint",
                       R=None, t=None):
    """RANSAC triangulation of track j (Sec. 4.3): hypothesis h = 0 .. n_hyp - 1 takes
    the observation pair ransac_pair(h, n) of the track (observations in index order),
    triangulates it by the midpoint of the two rays (triangulate_midpoint on the pair)
    and, when that succeeds, counts the track's observations with depth > Z_MIN and
    ||r|| <= tau_px at that point.  The first hypothesis with the most inliers wins; with
    at least two inliers the point is triangulated from them by ``method``.  Returns
    (X, ok, inlier flags over the track's observations)."""
    R = p.R if R is None else R
    t = p.t if t is None else t
    ks = np.nonzero(p.pt == j)[0]
    n = ks.size
    none = (None, False, np.zeros(n, bool))
    if n < 2:
        return none
    best, best_in = -1, None
    for h in range(n_hyp):
        a, b = ransac_pair(h, n)
        q = dataclasses.replace(p, active=np.zeros(p.n_obs, bool))
        q.active[[ks[a], ks[b]]] = True
        X, ok = triangulate_midpoint(q, j, R, t)
        if not ok:
            continue
        Kk = p.K[p.cam[ks]]
        uv, Pc = project(Kk, R[p.cam[ks]], t[p.cam[ks]], np.broadcast_to(X, (n, 3)))
        inl = (Pc[:, 2] > Z_MIN) & (np.sum((uv - p.uv[ks]) ** 2, axis=1) <= tau_px * tau_px)
        if int(inl.sum()) > best:
            best, best_in = int(inl.sum()), inl
    if best < 2:
        return none
    q = dataclasses.replace(p, active=np.zeros(p.n_obs, bool))
    q.active[ks[best_in]] = True
    X, ok = (triangulate_midpoint if method == "midpoint" else triangulate_dlt)(q, j, R, t)
    return (X, True, best_in) if ok else none
