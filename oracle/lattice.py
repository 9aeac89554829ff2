"""Sample positions of each field component on the rectilinear grid.

The paper sums eq:1 over every voxel and every polarization, the latter
"usually defined at staggered grid locations" (Sec. "Background"), and its
finite-difference baseline re-meshes once per Yee half-step (Sec.
"Polarization-splitting grating coupler in 3D").  It does not give the
offsets.  Reading used here (Yee): component E_a is sampled at the cell
center along axis a and at the cell's lower node along the other axes.

For a sample, its *averaging interval* along an axis is
[center - width/2, center + width/2]:
  cell-centered : center (A_i + A_{i+1})/2, width A_{i+1} - A_i
  node-centered : center A_i,  width (w_{i-1} + w_i)/2 with w_{-1} := w_0
for i = 0 .. N-1 (every component plane has N samples along each axis).
"""
import numpy as np

AXES = ("x", "y", "z")


def axis_samples(nodes, cell_centered):
    A = np.asarray(nodes, dtype=np.float64)
    w = A[1:] - A[:-1]
    if cell_centered:
        return 0.5 * (A[:-1] + A[1:]), w.copy()
    wl = np.concatenate([[w[0]], w[:-1]])
    return A[:-1].copy(), 0.5 * (wl + w)


def component_samples(scene, comp):
    """{axis: (centers, widths)} for component letter ``comp``."""
    out = {}
    for a, nodes in zip(AXES, scene["nodes"]):
        out[a] = axis_samples(nodes, cell_centered=(a == comp))
    return out
