"""Seeded synthetic proton phantoms: dose (D) and LET-weighted dose (L) influence
matrices plus per-voxel bounds, priorities and objective targets.

This module only builds inputs. It contains none of the optimizer's arithmetic:
no projections, no objective, no gradient. It is the single input source shared
by the FP64 oracle (in ``oracle/``) and the HIP path, so both see bit-identical
FP32 arrays.

Physics stand-ins (the paper's matrices come from FRED Monte Carlo on patient CTs,
which are not available; Section 2.2 describes what they hold):

* homogeneous water, straight rays, parallel pencil beams per field;
* D_ij = A * B(depth/R_j) * G(lateral distance), with a Gaussian lateral profile G
  cut at 3 sigma and a Bragg-peaked depth curve B(t) = (1 - 0.96 t)^(-1/2) for
  t <= 1, zero beyond the range R_j;
* LET_ij = 0.5 keV/um up to 90 % of the range, then rising linearly to 10 keV/um
  at the range; L_ij = D_ij * LET_ij.  LETd numerator and denominator are stored
  separately because only they are additive (Section 2.2, Eq. 1); the dose matrix
  serves as the denominator;
* A is chosen so the mean PTV dose at unit fluence is 2.0 Gy (74 Gy in 37
  fractions, Section 2.1).

Constraint encoding per voxel row (``kind`` bit mask), Fig. 2 and Eq. (2):
  DOSE_LO / DOSE_HI   lower / upper dose bound          (a = D_i)
  CDL_LO  / CDL_HI    lower / upper bound on c*dose*LETd (a = c L_i)
  LETD_HI             LETd_i <= T_i, linearised as (L_i - T_i D_i) x <= 0
  OBJ_DOSE            PTV term of Eq. (2):  w (Dhat - d_i)^2
  OBJ_CDL             OAR term of Eq. (2):  w (cDLhat - c l_i)^2
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

DOSE_LO = 1 << 0
DOSE_HI = 1 << 1
CDL_LO = 1 << 2
CDL_HI = 1 << 3
LETD_HI = 1 << 4
OBJ_DOSE = 1 << 5
OBJ_CDL = 1 << 6
CONSTRAINT_BITS = DOSE_LO | DOSE_HI | CDL_LO | CDL_HI | LETD_HI

C_DL = 0.04  # um/keV, Section 2.4 (Unkelbach et al. 2016)

PROBLEM_FIELDS = ("kind", "dose_lo", "dose_hi", "cdl_lo", "cdl_hi", "letd_max",
                  "w_feas", "w_obj", "dose_target", "cdl_target")


@dataclasses.dataclass
class Phantom:
    """CSR influence matrices with a shared sparsity pattern plus the per-row problem."""
    name: str
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray     # int64 [R+1]
    col_idx: np.ndarray     # int32 [nnz], strictly increasing within a row
    d_val: np.ndarray       # float32 [nnz], Gy per unit fluence
    l_val: np.ndarray       # float32 [nnz], Gy * keV/um per unit fluence
    kind: np.ndarray        # uint16 [R]
    dose_lo: np.ndarray     # float32 [R] (Gy)
    dose_hi: np.ndarray
    cdl_lo: np.ndarray      # float32 [R] (Gy, c*dose*LETd)
    cdl_hi: np.ndarray
    letd_max: np.ndarray    # float32 [R] (keV/um)
    w_feas: np.ndarray      # float32 [R], AMS priority w_i (Fig. 2)
    w_obj: np.ndarray       # float32 [R], Eq. (2) weight
    dose_target: np.ndarray  # float32 [R], Dhat_i
    cdl_target: np.ndarray   # float32 [R], cDLhat_i
    x0: np.ndarray          # float32 [C], initial fluence
    c: float = C_DL
    roi: Dict[str, np.ndarray] = dataclasses.field(default_factory=dict)
    meta: Dict[str, object] = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def problem_arrays(self) -> Dict[str, np.ndarray]:
        return {k: getattr(self, k) for k in PROBLEM_FIELDS}

    def dose_only(self) -> "Phantom":
        """The same plan with the paper's "dose only" problem (Section 2.5, the dose
        arms of Table 2): dose bounds and the PTV dose objective kept, every cDL and
        LETd constraint and the OAR cDL objective dropped.  The matrices are shared."""
        keep = np.uint16(DOSE_LO | DOSE_HI | OBJ_DOSE)
        return dataclasses.replace(self, name=f"{self.name}_dose_only",
                                   kind=(self.kind & keep).astype(np.uint16),
                                   meta={**self.meta, "problem": "dose only"})

    def summary(self) -> Dict[str, object]:
        return {"name": self.name, "rows": self.n_rows, "cols": self.n_cols,
                "nnz": self.nnz, **{k: v for k, v in self.meta.items()
                                    if isinstance(v, (int, float, str))}}


def _empty_problem(R: int) -> Dict[str, np.ndarray]:
    z = lambda: np.zeros(R, np.float32)  # noqa: E731
    return {"kind": np.zeros(R, np.uint16), "dose_lo": z(), "dose_hi": z(),
            "cdl_lo": z(), "cdl_hi": z(), "letd_max": z(),
            "w_feas": np.ones(R, np.float32), "w_obj": np.ones(R, np.float32),
            "dose_target": z(), "cdl_target": z()}


def percentile_nearest_rank(values: np.ndarray, q: float) -> float:
    """Value at 1-based rank ceil(q*n) of the ascending sort (q in (0,1])."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return 0.0
    k = max(1, int(math.ceil(q * v.size - 1e-12)))
    return float(v[k - 1])


# ----------------------------------------------------------------------------------
# tiny random problems (oracle pins, ragged parity cases)
# ----------------------------------------------------------------------------------

def random_sparse(R: int, C: int, density: float, seed: int, *,
                  empty_rows: Sequence[int] = (), empty_cols: Sequence[int] = (),
                  let_range: Tuple[float, float] = (0.5, 10.0)) -> Tuple[np.ndarray, ...]:
    """Random CSR (row_ptr, col, D, L) with D > 0 and L = D * LET, LET uniform."""
    rng = np.random.default_rng(seed)
    mask = rng.random((R, C)) < density
    if R and C:
        # every non-forced-empty row gets at least one entry
        for i in range(R):
            if not mask[i].any():
                mask[i, rng.integers(C)] = True
    for i in empty_rows:
        mask[i, :] = False
    for j in empty_cols:
        mask[:, j] = False
    rows, cols = np.nonzero(mask)
    nnz = rows.size
    d = rng.uniform(0.05, 1.0, nnz).astype(np.float32)
    let = rng.uniform(let_range[0], let_range[1], nnz).astype(np.float32)
    l = (d * let).astype(np.float32)
    row_ptr = np.zeros(R + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=R), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), d, l


def tiny_problem(R: int = 48, C: int = 12, density: float = 0.3, seed: int = 0, *,
                 empty_rows: Sequence[int] = (), empty_cols: Sequence[int] = (),
                 let_range: Tuple[float, float] = (0.5, 10.0),
                 kinds: str = "mixed") -> Phantom:
    """A small random problem whose bounds straddle the dose at x0 = 1, so that some
    rows of every constraint kind are violated and some are not."""
    rng = np.random.default_rng(seed + 7919)
    row_ptr, col, d, l = random_sparse(R, C, density, seed, empty_rows=empty_rows,
                                       empty_cols=empty_cols, let_range=let_range)
    x0 = np.ones(C, np.float32)
    # row sums at x0 = 1, used only to place bounds around the starting point
    rid = np.repeat(np.arange(R), np.diff(row_ptr))
    d0 = np.bincount(rid, weights=d.astype(np.float64), minlength=R)
    l0 = np.bincount(rid, weights=l.astype(np.float64), minlength=R)
    p = _empty_problem(R)
    kind = np.zeros(R, np.uint16)
    third = max(1, R // 3)
    for i in range(R):
        u = rng.random()
        if kinds == "dose" or (kinds == "mixed" and i < third):
            kind[i] = DOSE_LO | DOSE_HI | OBJ_DOSE
            p["dose_lo"][i] = d0[i] * rng.uniform(0.8, 1.1)
            p["dose_hi"][i] = max(p["dose_lo"][i], d0[i] * rng.uniform(0.9, 1.3))
            p["dose_target"][i] = d0[i] * rng.uniform(0.9, 1.1)
        elif kinds == "mixed" and i < 2 * third:
            kind[i] = DOSE_HI | LETD_HI | OBJ_CDL
            p["dose_hi"][i] = d0[i] * rng.uniform(0.7, 1.2)
            letd = l0[i] / d0[i] if d0[i] > 0 else 1.0
            p["letd_max"][i] = letd * rng.uniform(0.8, 1.2)
            p["cdl_target"][i] = C_DL * l0[i] * rng.uniform(0.5, 1.0)
        else:
            kind[i] = CDL_LO | CDL_HI
            c0 = C_DL * l0[i]
            p["cdl_lo"][i] = c0 * rng.uniform(0.8, 1.1)
            p["cdl_hi"][i] = max(p["cdl_lo"][i], c0 * rng.uniform(0.9, 1.3))
        p["w_feas"][i] = rng.uniform(0.5, 2.0)
        p["w_obj"][i] = rng.uniform(0.5, 2.0)
        del u
    p["kind"] = kind
    return Phantom(name=f"tiny_R{R}_C{C}_s{seed}", n_rows=R, n_cols=C, row_ptr=row_ptr,
                   col_idx=col, d_val=d, l_val=l, x0=x0, c=C_DL,
                   roi={"all": np.arange(R)}, meta={"seed": seed}, **p)


# ----------------------------------------------------------------------------------
# geometric water phantoms (configs of the hot-path workloads)
# ----------------------------------------------------------------------------------

def bragg_depth(t: np.ndarray) -> np.ndarray:
    """Relative depth dose at fractional depth t = depth / range (t <= 1)."""
    return 1.0 / np.sqrt(1.0 - 0.96 * t)


def let_depth(t: np.ndarray) -> np.ndarray:
    """LET (keV/um) at fractional depth t: 0.5 up to 0.9, linear to 10 at t = 1."""
    return np.where(t <= 0.9, 0.5, 0.5 + (t - 0.9) * (9.5 / 0.1))


@dataclasses.dataclass
class Field:
    gantry_deg: float                  # beam direction in the x-y plane
    n_u: int                           # spots along the in-plane lateral axis
    n_v: int                           # spots along z
    span_u_mm: float                   # lateral extent covered by spot centres
    span_v_mm: float


def _box_depth(pos: np.ndarray, b: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Distance from the entry face of the box [0, box] to each point, travelling
    along direction b (straight rays in homogeneous water)."""
    depth = np.full(pos.shape[0], np.inf, np.float64)
    for k in range(3):
        if b[k] > 1e-12:
            depth = np.minimum(depth, pos[:, k] / b[k])
        elif b[k] < -1e-12:
            depth = np.minimum(depth, (box[k] - pos[:, k]) / (-b[k]))
    return depth


def beam_matrices(shape: Tuple[int, int, int], h_mm: float, iso_mm: np.ndarray,
                  fields: List[Field], sigma_mm: float, ranges_mm: np.ndarray,
                  keep_all: bool = False, progress: Optional[Callable[[str], None]] = None):
    """CSR (voxels x beamlets) of D and LET for parallel pencil beams in a water box.

    Columns are ordered field, then spot row (v), then spot column (u), so that for a
    fixed voxel the window scan below emits columns in increasing order and the CSR
    needs no sort. Returns (voxel_ids_of_rows, row_ptr, col, D_unnormalised, LET).
    """
    nx, ny, nz = shape
    box = np.array([nx, ny, nz], np.float64) * h_mm
    n_vox = nx * ny * nz
    cut2 = (3.0 * sigma_mm) ** 2
    passes = []   # (vox ids int64, cols int32 [n, w], D f32 [n, w], LET f32 [n,w], valid [n, w])
    counts = np.zeros(n_vox, np.int64)
    col_base = 0
    rmax = float(np.max(ranges_mm)) if len(ranges_mm) else 0.0
    for fi, f in enumerate(fields):
        th = math.radians(f.gantry_deg)
        b = np.array([math.cos(th), math.sin(th), 0.0])
        u = np.array([-math.sin(th), math.cos(th), 0.0])
        v = np.array([0.0, 0.0, 1.0])
        du = f.span_u_mm / max(1, f.n_u - 1)
        dv = f.span_v_mm / max(1, f.n_v - 1)
        u0 = -0.5 * f.span_u_mm
        v0 = -0.5 * f.span_v_mm
        # candidate voxels: inside the lateral footprint of the spot grid
        zc = (np.arange(nz) + 0.5) * h_mm
        yc = (np.arange(ny) + 0.5) * h_mm
        xc = (np.arange(nx) + 0.5) * h_mm
        Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
        pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        rel = pos - iso_mm[None, :]
        pu = rel @ u
        pv = rel @ v
        marg = 3.0 * sigma_mm + max(du, dv)
        sel = ((pu >= u0 - marg) & (pu <= -u0 + marg) & (pv >= v0 - marg) & (pv <= -v0 + marg))
        vid = np.nonzero(sel)[0].astype(np.int64)
        depth = _box_depth(pos[vid], b, box)
        keep = depth <= rmax
        vid, depth = vid[keep], depth[keep]
        pu, pv = pu[vid], pv[vid]
        del pos, rel, X, Y, Z
        ka = int(math.ceil(3.0 * sigma_mm / du)) + 1 if f.n_u > 1 else 0
        kb = int(math.ceil(3.0 * sigma_mm / dv)) + 1 if f.n_v > 1 else 0
        a_c = np.rint((pu - u0) / du).astype(np.int64) if f.n_u > 1 else np.zeros(vid.size, np.int64)
        b_c = np.rint((pv - v0) / dv).astype(np.int64) if f.n_v > 1 else np.zeros(vid.size, np.int64)
        da = np.arange(-ka, ka + 1, dtype=np.int64)
        ns = f.n_u * f.n_v
        rng_f = ranges_mm[col_base:col_base + ns]
        for db in range(-kb, kb + 1):
            bb = b_c + db
            okb = (bb >= 0) & (bb < f.n_v)
            idx = np.nonzero(okb)[0]
            if idx.size == 0:
                continue
            bbv = bb[idx]
            ddv = pv[idx] - (v0 + bbv * dv)
            aa = a_c[idx, None] + da[None, :]
            ok = (aa >= 0) & (aa < f.n_u)
            ddu = pu[idx, None] - (u0 + aa * du)
            r2 = ddu * ddu + (ddv * ddv)[:, None]
            ok &= r2 <= cut2
            spot = bbv[:, None] * f.n_u + np.clip(aa, 0, f.n_u - 1)
            R_j = rng_f[spot]
            t = depth[idx, None] / R_j
            ok &= t <= 1.0
            rows_ok = ok.any(axis=1)
            if not rows_ok.any():
                continue
            ii = np.nonzero(rows_ok)[0]
            ok = ok[ii]
            tt = np.where(ok, t[ii], 0.0)
            g = np.exp(-r2[ii] / (2.0 * sigma_mm * sigma_mm))
            dval = (bragg_depth(tt) * g).astype(np.float32)
            letv = let_depth(tt).astype(np.float32)
            cols = (col_base + spot[ii]).astype(np.int32)
            vv = vid[idx[ii]]
            counts[vv] += ok.sum(axis=1)
            passes.append((vv, cols, dval, letv, ok))
        col_base += ns
        if progress:
            progress(f"field {fi}: {sum(int(p[4].sum()) for p in passes)} nnz so far")
    if keep_all:
        kept = np.arange(n_vox, dtype=np.int64)
    else:
        kept = np.nonzero(counts)[0].astype(np.int64)
    row_of = np.full(n_vox, -1, np.int64)
    row_of[kept] = np.arange(kept.size)
    R = kept.size
    row_ptr = np.zeros(R + 1, np.int64)
    np.cumsum(counts[kept], out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, np.int32)
    dv_out = np.empty(nnz, np.float32)
    let_out = np.empty(nnz, np.float32)
    cursor = row_ptr[:-1].copy()
    for vv, cols, dval, letv, ok in passes:
        r = row_of[vv]
        rank = np.cumsum(ok, axis=1) - 1
        pos = cursor[r][:, None] + rank
        col[pos[ok]] = cols[ok]
        dv_out[pos[ok]] = dval[ok]
        let_out[pos[ok]] = letv[ok]
        cursor[r] += ok.sum(axis=1)
    assert np.array_equal(cursor, row_ptr[1:])
    return kept, row_ptr, col, dv_out, let_out


def _voxel_centres(shape, h_mm, vox_ids):
    nx, ny, nz = shape
    x = vox_ids % nx
    y = (vox_ids // nx) % ny
    z = vox_ids // (nx * ny)
    return np.stack([(x + 0.5) * h_mm, (y + 0.5) * h_mm, (z + 0.5) * h_mm], axis=1)


def _finish(name, shape, h_mm, kept, row_ptr, col, d_raw, let, C, masks, bounds, seed,
            extra_meta=None, dose_scale: Optional[float] = None) -> Phantom:
    """Normalise dose, build L = D * LET and the per-row problem.  dose_scale: the
    factor that turns raw depth-dose into Gy per unit fluence, given for a robustness
    scenario (the nominal plan's), else chosen so that the mean PTV dose at unit
    fluence is 2 Gy."""
    R = kept.size
    ptv = masks["PTV"]
    d_raw64 = d_raw.astype(np.float64)
    rid = np.repeat(np.arange(R), np.diff(row_ptr))
    rs = np.bincount(rid, weights=d_raw64, minlength=R)
    if dose_scale is not None:
        A = float(dose_scale)
    else:
        A = 2.0 / float(np.mean(rs[ptv])) if ptv.any() else 1.0
    d = (d_raw64 * A).astype(np.float32)
    l = (d.astype(np.float64) * let.astype(np.float64)).astype(np.float32)
    # row sums at unit fluence of the stored FP32 values: place the OAR cDL target
    lsum = np.bincount(rid, weights=l.astype(np.float64), minlength=R)
    p = _empty_problem(R)
    kind = np.zeros(R, np.uint16)
    lo, hi, rx = bounds["ptv_lo"], bounds["ptv_hi"], bounds["rx"]
    kind[ptv] = DOSE_LO | DOSE_HI | OBJ_DOSE
    p["dose_lo"][ptv] = lo
    p["dose_hi"][ptv] = hi
    p["dose_target"][ptv] = rx
    oar_all = np.zeros(R, bool)
    for name_o, m in masks.items():
        if not name_o.startswith("OAR"):
            continue
        m = m & ~ptv
        oar_all |= m
        kind[m] = DOSE_HI | LETD_HI | OBJ_CDL
        p["dose_hi"][m] = bounds["oar_dose_hi"]
        p["letd_max"][m] = bounds["oar_letd_max"]
        cdl30 = percentile_nearest_rank(C_DL * lsum[m], 0.70) if m.any() else 0.0
        p["cdl_target"][m] = cdl30
    if "normal_dose_hi" in bounds:
        rest = ~ptv & ~oar_all
        kind[rest] = DOSE_HI
        p["dose_hi"][rest] = bounds["normal_dose_hi"]
    p["kind"] = kind
    roi = {k: np.nonzero(v)[0] for k, v in masks.items()}
    meta = {"seed": seed, "grid": "x".join(map(str, shape)), "voxel_mm": h_mm,
            "dose_scale": A, **(extra_meta or {})}
    return Phantom(name=name, n_rows=R, n_cols=C, row_ptr=row_ptr, col_idx=col,
                   d_val=d, l_val=l, x0=np.ones(C, np.float32), c=C_DL, roi=roi,
                   meta=meta, **p)


def water32(seed: int = 0) -> Phantom:
    """Tiny phantom: 32^3 water grid at 3 mm, all voxels kept; two opposed fields
    along +-x with a 20 x 10 spot grid each (400 beamlets); sigma 1.5 voxels cut at
    3 sigma; ranges U[30, 80] mm; spherical PTV (r = 8 voxels, centre) bounded to
    1.9-2.14 Gy; cylindrical OAR (r = 3 voxels, axis along z) just distal to the
    PTV for the +x field with dose <= 1.0 Gy and LETd <= 2 keV/um."""
    shape, h = (32, 32, 32), 3.0
    rng = np.random.default_rng(seed)
    iso = np.array([48.0, 48.0, 48.0])
    sigma = 1.5 * h
    r_ptv = 8 * h
    span_u = 2 * (r_ptv + sigma)
    fields = [Field(0.0, 20, 10, span_u, span_u), Field(180.0, 20, 10, span_u, span_u)]
    C = 400
    ranges = rng.uniform(30.0, 80.0, C)
    kept, row_ptr, col, d_raw, let = beam_matrices(shape, h, iso, fields, sigma, ranges,
                                                   keep_all=True)
    p = _voxel_centres(shape, h, kept)
    ptv = np.sum((p - iso) ** 2, axis=1) <= r_ptv ** 2
    oar = ((p[:, 0] - 28.5 * h) ** 2 + (p[:, 1] - 16.5 * h) ** 2) <= (3 * h) ** 2
    masks = {"PTV": ptv, "OAR_cyl": oar & ~ptv}
    bounds = {"ptv_lo": 1.9, "ptv_hi": 2.14, "rx": 2.0, "oar_dose_hi": 1.0,
              "oar_letd_max": 2.0}
    return _finish("water32_400beamlets", shape, h, kept, row_ptr, col, d_raw, let, C,
                   masks, bounds, seed, {"iterations": 100, "sigma_mm": sigma})


def clinical(seed: int = 1, progress: Optional[Callable[[str], None]] = None,
            scale: float = 1.0) -> Phantom:
    """Clinical-scale phantom: 160 x 160 x 120 grid at 2 mm; three coplanar fields
    (0, 120, 240 degrees) with an 80 x 50 spot grid each (12,000 beamlets); ranges
    U[50, 200] mm; every irradiated voxel is a row.  Ellipsoidal PTV with diameters
    6 x 5 x 5 cm at the centre, a brainstem-like cylinder and a chiasm-like slab as
    OARs (dose <= 1 Gy, LETd <= 2 keV/um), every other kept voxel carries a
    normal-tissue dose upper bound of 2.14 Gy.  ``scale`` < 1 shrinks the grid and
    spot counts proportionally (for quick tests)."""
    h = 2.0
    shape = tuple(int(round(n * scale)) for n in (160, 160, 120))
    rng = np.random.default_rng(seed)
    box = np.array(shape, np.float64) * h
    iso = box / 2.0
    sigma = 2.7 * h
    nu, nv = max(2, int(round(80 * scale))), max(2, int(round(50 * scale)))
    semi = np.array([30.0, 25.0, 25.0]) * scale
    span_u, span_v = 2 * semi[0], 2 * semi[2]
    fields = [Field(g, nu, nv, span_u, span_v) for g in (0.0, 120.0, 240.0)]
    C = 3 * nu * nv
    ranges = rng.uniform(50.0 * scale, 200.0 * scale, C)
    kept, row_ptr, col, d_raw, let = beam_matrices(shape, h, iso, fields, sigma, ranges,
                                                   progress=progress)
    p = _voxel_centres(shape, h, kept) - iso
    ptv = np.sum((p / semi) ** 2, axis=1) <= 1.0
    # brainstem-like cylinder (r = 12.5 mm, axis along z) behind the PTV along -y
    bs_r = 12.5 * scale
    bs_c = np.array([0.0, -(semi[1] + bs_r + 2.0 * scale)])
    brainstem = ((p[:, 0] - bs_c[0]) ** 2 + (p[:, 1] - bs_c[1]) ** 2 <= bs_r ** 2) & \
        (np.abs(p[:, 2]) <= 30.0 * scale)
    # chiasm-like slab above the PTV (+z), 30 x 14 x 4 mm
    chiasm = (np.abs(p[:, 0]) <= 15.0 * scale) & (np.abs(p[:, 1] - 5.0 * scale) <= 7.0 * scale) & \
        (p[:, 2] >= semi[2] + 2.0 * scale) & (p[:, 2] <= semi[2] + 6.0 * scale)
    masks = {"PTV": ptv, "OAR_brainstem": brainstem & ~ptv, "OAR_chiasm": chiasm & ~ptv & ~brainstem}
    bounds = {"ptv_lo": 1.9, "ptv_hi": 2.14, "rx": 2.0, "oar_dose_hi": 1.0,
              "oar_letd_max": 2.0, "normal_dose_hi": 2.14}
    return _finish("clinical_160x160x120_12k" if scale == 1.0 else f"clinical_scaled_{scale:g}",
                   shape, h, kept, row_ptr, col, d_raw, let, C, masks, bounds, seed,
                   {"iterations": 1000, "sigma_mm": sigma})


def small_plan(seed: int, n_rows_target: int, n_cols_target: int, range_scale: float = 1.0,
               shift_mm: Sequence[float] = (0.0, 0.0, 0.0), tag: str = "",
               dose_scale: Optional[float] = None) -> Phantom:
    """One plan of the batched workload: a cubic water grid holding about
    n_rows_target voxels (all kept), two opposed fields with n_cols_target/2 spots
    each, the density of the 32^3 water phantom (sigma 1.5 voxels, 3 mm voxels, ranges
    spanning 30-90 % of the grid depth).

    Robustness scenarios of the same plan: range_scale multiplies every beamlet
    range (a stopping-power error), shift_mm moves the beams against the patient (a
    setup error); structures, bounds and targets stay where the nominal plan has
    them."""
    rng = np.random.default_rng(seed)
    n = max(8, int(round(n_rows_target ** (1.0 / 3.0))))
    shape, h = (n, n, n), 3.0
    iso = np.array([n * h / 2] * 3)
    sigma = 1.5 * h
    r_ptv = max(2.0, n / 4.0) * h
    half = max(1, n_cols_target // 2)
    nv = max(1, int(round(math.sqrt(half / 2.0))))
    nu = max(1, half // nv)
    span = 2 * (r_ptv + sigma)
    fields = [Field(0.0, nu, nv, span, span), Field(180.0, nu, nv, span, span)]
    C = 2 * nu * nv
    depth = n * h
    ranges = rng.uniform(0.3 * depth, 0.9 * depth, C) * float(range_scale)
    beam_iso = iso + np.asarray(shift_mm, np.float64)
    kept, row_ptr, col, d_raw, let = beam_matrices(shape, h, beam_iso, fields, sigma, ranges,
                                                   keep_all=True)
    p = _voxel_centres(shape, h, kept)
    ptv = np.sum((p - iso) ** 2, axis=1) <= r_ptv ** 2
    oar_x = iso[0] + r_ptv + 4 * h
    oar = ((p[:, 0] - oar_x) ** 2 + (p[:, 1] - iso[1]) ** 2) <= (max(1.0, n / 10.0) * h) ** 2
    masks = {"PTV": ptv, "OAR_cyl": oar & ~ptv}
    bounds = {"ptv_lo": 1.9, "ptv_hi": 2.14, "rx": 2.0, "oar_dose_hi": 1.0,
              "oar_letd_max": 2.0}
    return _finish(f"plan_s{seed}_{n}cube_C{C}{tag}", shape, h, kept, row_ptr, col, d_raw, let,
                   C, masks, bounds, seed, {"iterations": 100, "range_scale": float(range_scale),
                                            "shift_mm": [float(v) for v in shift_mm]},
                   dose_scale=dose_scale)


# range errors and setup shifts of the robustness scenarios (8 per base plan)
SCENARIOS = [(1.035, (0.0, 0.0, 0.0)), (0.965, (0.0, 0.0, 0.0)),
             (1.0, (3.0, 0.0, 0.0)), (1.0, (-3.0, 0.0, 0.0)),
             (1.0, (0.0, 3.0, 0.0)), (1.0, (0.0, -3.0, 0.0)),
             (1.0, (0.0, 0.0, 3.0)), (1.0, (0.0, 0.0, -3.0))]


def scenario_plans(n_base: int = 6, seed: int = 3) -> List[Phantom]:
    """n_base plans of the batched workload (the first draws), each regenerated from
    the same seed under the eight robustness scenarios: ranges x (1 +- 3.5 %) and
    +-3 mm setup shifts along each axis."""
    out = []
    for sd, r, c in batch_sizes(n_base, seed):
        for k, (rs, sh) in enumerate(SCENARIOS):
            out.append(small_plan(sd, r, c, range_scale=rs, shift_mm=sh, tag=f"_sc{k}"))
    return out


def robustness_scenarios(seed: int, n_rows_target: int, n_cols_target: int,
                         shift_mm: float = 2.0, range_error: float = 0.035) -> List[Phantom]:
    """The nominal plan and the recalculations of its robustness evaluation (Section
    2.5: +-2 mm setup shifts along each axis and +-3.5 % density, 9 in all): beamlet
    ranges scaled by 1 -+ range_error (denser water stops the beam earlier) and the
    beams shifted against the patient.  Every scenario keeps the nominal plan's voxel
    rows (all voxels of the same grid), beamlets and dose scale, so row i is the same
    voxel and column j the same beamlet throughout."""
    nominal = small_plan(seed, n_rows_target, n_cols_target, tag="_nominal")
    A = float(nominal.meta["dose_scale"])
    out = [nominal]
    for k, rs in enumerate((1.0 - range_error, 1.0 + range_error)):
        out.append(small_plan(seed, n_rows_target, n_cols_target, range_scale=rs,
                              tag=f"_range{k}", dose_scale=A))
    for axis in range(3):
        for sign in (1.0, -1.0):
            sh = [0.0, 0.0, 0.0]
            sh[axis] = sign * shift_mm
            out.append(small_plan(seed, n_rows_target, n_cols_target, shift_mm=sh,
                                  tag=f"_shift{axis}{'p' if sign > 0 else 'm'}", dose_scale=A))
    return out


def batch_sizes(n_plans: int = 48, seed: int = 3) -> List[Tuple[int, int, int]]:
    """(seed, rows, beamlets) of the batched workload: one u ~ U[0,1] per plan maps
    log-uniformly to both rows (5k-120k) and beamlets (200-4,000)."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(n_plans):
        u = rng.random()
        rows = int(round(math.exp(math.log(5e3) + u * (math.log(1.2e5) - math.log(5e3)))))
        cols = int(round(math.exp(math.log(200) + u * (math.log(4000) - math.log(200)))))
        out.append((3000 + p, rows, cols))
    return out
