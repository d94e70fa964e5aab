"""Writes closed_form.json: expected values derived from the paper's equations by hand.

Cases (literal mode: no alpha clamp, skip or termination):
* an isotropic Gaussian (scale s, opacity o, colour c) at camera-space point t seen by a
  pinhole camera with R_cw = I: mu' = f t_xy / t_z + c_xy + 1/2 (eqs. 1-2), Sigma' =
  s^2 J J^T with J of eq. (3); the pixel value is c o exp(-1/2 Delta^T Sigma'^{-1} Delta)
  with Delta = mu' - pixel centre (eq. 7 with one Gaussian);
* two Gaussians on the optical axis, the nearer one composited first:
  C = c1 a1 + c2 a2 (1 - a1) and T = (1 - a1)(1 - a2) (eq. 7).
"""
import json
import os

import numpy as np


def single(fx, fy, cx, cy, t, s, o, c, pixels):
    t = np.asarray(t, dtype=np.float64)
    J = np.array([[fx / t[2], 0, -fx * t[0] / t[2] ** 2], [0, fy / t[2], -fy * t[1] / t[2] ** 2]])
    cov = s * s * J @ J.T
    Y = np.linalg.inv(cov)
    mu = np.array([fx * t[0] / t[2] + cx + 0.5, fy * t[1] / t[2] + cy + 0.5])
    vals = []
    for (i, j) in pixels:
        d = mu - np.array([j + 0.5, i + 0.5])
        a = o * np.exp(-0.5 * d @ Y @ d)
        vals.append([ci * a for ci in c] + [1 - a])
    return {"mean2d": mu.tolist(), "cov2d": cov.tolist(), "pixels": pixels, "rgb_T": vals}


def main():
    f32 = lambda x: float(np.float32(x))
    cases = []
    s, o, c = f32(0.08), f32(0.7), [f32(0.2), f32(0.5), f32(0.9)]
    t = [f32(0.1), f32(-0.05), 3.0]
    cases.append({"kind": "single", "camera": {"fx": 64.0, "fy": 64.0, "cx": 32.0, "cy": 32.0, "W": 64, "H": 64},
                  "mean": t, "scale": s, "opacity": o, "color": c,
                  "expected": single(64.0, 64.0, 32.0, 32.0, t, s, o, c, [[32, 34], [30, 33], [35, 31]])})
    o1, o2 = f32(0.6), f32(0.8)
    cases.append({"kind": "stacked", "camera": {"fx": 64.0, "fy": 64.0, "cx": 32.0, "cy": 32.0, "W": 64, "H": 64},
                  "depths": [2.0, 4.0], "opacities": [o1, o2], "colors": [[1.0, 0.0, 0.5], [0.0, 1.0, 0.25]],
                  "pixel": [32, 32],
                  "expected_rgb": [1.0 * o1 + 0.0, 0.0 + 1.0 * o2 * (1 - o1), 0.5 * o1 + 0.25 * o2 * (1 - o1)],
                  "expected_T": (1 - o1) * (1 - o2)})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_form.json")
    with open(path, "w") as fh:
        json.dump({"source": "gsplat supplement eqs. (1)-(3), (7); values derived by hand", "cases": cases}, fh,
                  indent=1)


if __name__ == "__main__":
    main()
