"""MI355X (gfx950) tile-based differentiable tetrahedron rasterizer of
"Tetrahedron Splatting for 3D Generation" (TeT-Splatting, arXiv 2406.01579).

The rendering runs in hand-written HIP kernels behind the C ABI of
include/tetsplat.h (libtetsplat.so, built in-tree by
``python -m paper_2406_01579_amd.build``).  This package is the thin Python
side: argument marshalling, workspace sizing and ownership, and a
torch.autograd.Function.
"""
from .frontend import CapacityError, Params, Plan, Renderer, SceneT, TetSplatFunction, render  # noqa: F401
from .graph import CapturedStep  # noqa: F401
