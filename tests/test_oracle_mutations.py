"""Planted-mistake sweep: each mutation below plants one plausible mistake
(a dropped term, a wrong sign, index or constant, a transposed operand) in a
copy of the oracle, and the oracle's pins (tests/test_oracle_*.py, run in a
child process against that copy) must fail.  The unmutated copy must pass.
The HIP path is not involved."""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
              if f.startswith("test_oracle_") and f.endswith(".py") and f != "test_oracle_mutations.py")

# (file in oracle/, original text, planted text, what it stands for)
MUTATIONS = [
    ("raster.py", "ALPHA_MAX = 0.99", "ALPHA_MAX = 0.95", "wrong opacity clamp"),
    ("raster.py", "ALPHA_MIN = 1.0 / 255.0", "ALPHA_MIN = 1.0 / 128.0", "wrong skip threshold"),
    ("raster.py", "T_STOP = 1e-4", "T_STOP = 1e-3", "wrong stop threshold"),
    ("raster.py", "Q_MAX = 9.0", "Q_MAX = 6.25", "2.5 sigma cut instead of 3 sigma"),
    ("raster.py", "incl = active & (t_after >= T_STOP)", "incl = active", "never stops"),
    ("raster.py", "t_after = torch.cumprod(1.0 - a_act, dim=1)",
     "t_after = torch.cat([torch.ones(P, 1, dtype=F64), torch.cumprod(1.0 - a_act, dim=1)[:, :-1]], 1) if L > 0 "
     "else torch.cumprod(1.0 - a_act, dim=1)", "adds the stopping Gaussian, then stops"),
    ("raster.py", "q = (conic[None, :, 0] * dx * dx + 2.0 * conic[None, :, 1] * dx * dy)",
     "q = (conic[None, :, 0] * dx * dx + conic[None, :, 1] * dx * dy)", "conic off-diagonal counted once"),
    ("raster.py", "px = pit.to(F64)[:, None] + 0.5", "px = pit.to(F64)[:, None]", "pixel corner instead of centre"),
    ("raster.py", "out_rgb = C + T[:, None] * torch.as_tensor(bg, dtype=F64)[None, :]", "out_rgb = C",
     "background dropped"),
    ("raster.py", "order = np.lexsort((gid, db, tid))", "order = np.lexsort((-gid, db, tid))",
     "equal depths ordered by descending index"),
    ("raster.py", "            if (a < ALPHA_MIN) != ((pos, \"a\") in flips):",
     "            if a < ALPHA_MIN:", "ambiguity variants ignore the alpha branch"),
    ("raster.py", "            if (Tn < T_STOP) != ((pos, \"t\") in flips):",
     "            if Tn < T_STOP:", "ambiguity variants ignore the stop branch"),
    ("project.py", "ca = c2[0][0] + cfg.dilation", "ca = c2[0][0]", "dilation dropped on one axis"),
    ("project.py", "1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),",
     "1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z + w * y),", "rotation sign"),
    ("project.py", "rx = 3.0 * torch.sqrt(torch.clamp(ca, min=0.0))", "rx = 2.5 * torch.sqrt(torch.clamp(ca, min=0.0))",
     "2.5 sigma box"),
    ("project.py", "xc = torch.clamp(xr, -limx, limx)", "xc = xr", "Jacobian clamp dropped"),
    ("project.py", "j02 = (-fx * xc) / safe_tz", "j02 = (fx * xc) / safe_tz", "Jacobian sign"),
    ("project.py", "conic = torch.stack([cc / safe_det, -cb / safe_det, ca / safe_det], dim=-1)",
     "conic = torch.stack([ca / safe_det, -cb / safe_det, cc / safe_det], dim=-1)", "conic diagonal swapped"),
    ("project.py", "Tm0 = [j00 * Rc[0, k] + j02 * Rc[2, k] for k in range(3)]",
     "Tm0 = [j00 * Rc[k, 0] + j02 * Rc[k, 2] for k in range(3)]", "camera rotation transposed"),
    ("project.py", "raw = (Y[:, :, None] * shk).sum(1) + 0.5", "raw = (Y[:, :, None] * shk).sum(1)",
     "colour offset dropped"),
    ("project.py", "rgb = torch.clamp(raw, min=0.0)", "rgb = raw", "colour clamp dropped"),
    ("project.py", "campos = [-((Rc[0, k] * tc[0] + Rc[1, k] * tc[1]) + Rc[2, k] * tc[2]) for k in range(3)]",
     "campos = [((Rc[0, k] * tc[0] + Rc[1, k] * tc[1]) + Rc[2, k] * tc[2]) for k in range(3)]",
     "camera centre sign"),
    ("project.py", 'for k in ("xy", "conic", "rgb", "depth", "opacity"):', 'for k in ("xy", "rgb", "depth", "opacity"):',
     "conic not rounded at the precision boundary"),
    ("sh.py", "row[l + m] = math.sqrt(2.0) * k * pz * re[m]", "row[l + m] = k * pz * re[m]",
     "SH normalisation of m > 0"),
    ("sh.py", "row[l - m] = math.sqrt(2.0) * k * pz * im[m]", "row[l - m] = math.sqrt(2.0) * k * pz * re[m]",
     "SH sine term replaced by the cosine term"),
    ("decoder.py", "loss = r.abs().sum() / P", "loss = r.abs().sum() / (P * C)", "loss averaged over channels too"),
    ("decoder.py", "d_feat=(Wt.T @ s)", "d_feat=(Wt.T @ (r / P))", "L2 gradient instead of the L1 subgradient"),
    ("decoder.py", "dec = Wt @ zf + b[:, None]", "dec = Wt @ zf", "decoder bias dropped"),
    ("decoder.py", "d_weight=(s @ zf.T)", "d_weight=(s @ zf.T).T.T * 0.5", "weight gradient halved"),
    ("deform.py", "PLANE_PAIRS = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))",
     "PLANE_PAIRS = ((0, 1), (0, 3), (0, 2), (1, 2), (1, 3), (2, 3))", "HexPlane pairs out of order"),
    ("deform.py", "wx * (1 - wy) * g[y0, x0 + 1]", "wx * (1 - wy) * g[y0 + 1, x0]", "bilinear taps transposed"),
    ("deform.py", "x = (ua + 1.0) / 2.0 * (ra - 1)", "x = (ua + 1.0) / 2.0 * ra", "grid end points off the box"),
    ("deform.py", "2.0 * float(t) - 1.0", "float(t)", "time not mapped to [-1, 1]"),
    ("deform.py", "prod = s if prod is None else prod * s", "prod = s if prod is None else prod + s",
     "planes summed instead of multiplied"),
    ("deform.py", "return base[coord] * level_mult if coord < 3 else base[coord]", "return base[coord] * level_mult",
     "time resolution refined with the levels"),
    ("deform.py", "x = _affine(x if i == 0 else torch.relu(x), layer)", "x = _affine(x, layer)",
     "no ReLU between the decoder layers"),
    ("deform.py", "u_all = torch.cat(hg, 1)", "u_all = torch.cat(hg[::-1], 1)", "branch features concatenated reversed"),
    ("deform.py", "opacity=torch.sigmoid(T(logit_opacity) + r[\"d_opacity\"][:, 0])",
     "opacity=torch.sigmoid(T(logit_opacity)) + r[\"d_opacity\"][:, 0]", "opacity update after the activation"),
]


def _run_pins(alt_root):
    env = dict(os.environ, FE_ORACLE_ROOT=alt_root, OMP_NUM_THREADS="1", PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def _copy_oracle(dst):
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__"))


def _mutant(args):
    fname, old, new, what = args
    with tempfile.TemporaryDirectory() as tmp:
        _copy_oracle(tmp)
        path = os.path.join(tmp, "oracle", fname)
        src = open(path).read()
        assert src.count(old) == 1, (fname, old)
        open(path, "w").write(src.replace(old, new))
        rc, out = _run_pins(tmp)
    return what, rc, out


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        _copy_oracle(tmp)
        rc, out = _run_pins(tmp)
    assert rc == 0, "the unmutated oracle copy must pass its pins:\n" + out
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(_mutant, MUTATIONS))
    survivors = [what for what, rc, _ in results if rc == 0]
    errors = [(what, out) for what, rc, out in results if rc not in (0, 1)]
    assert not errors, errors
    assert not survivors, f"planted mistakes no pin caught: {survivors}"
