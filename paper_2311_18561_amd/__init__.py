"""MI355X-native (gfx950) PVG splatting rasterizer.

The differentiable tile-based renderer of Periodic Vibration Gaussian
(arXiv 2311.18561): time-dependent means and opacities (Sec. 3.2), EWA
projection and alpha blending (Sec. 3.1), flow-translated second render
(Sec. 3.4), a hand-written adjoint, and a continuous-batching render server.
All computation runs in ``libpvg.so`` (HIP kernels behind a C ABI declared in
``include/pvg.h``); this package only marshals arguments and borrows PyTorch's
device memory and streams.
"""
from ._lib import PVGError, load  # noqa: F401
from .densify import densify, densify_config, split_by_staticness  # noqa: F401
from .optim import SKY_LR, DenseAdam, PVGAdam, default_lrs  # noqa: F401
from .scene_io import load_scene, save_scene  # noqa: F401
from .train import temporal_smoothing_views  # noqa: F401
from .render import (  # noqa: F401
    FIELDS,
    PVGRender,
    PVGRenderViews,
    PVGSkyComposite,
    bin_sort,
    bin_sort_nosync,
    camera_struct,
    frame_struct,
    preprocess,
    preprocess_views,
    pvg_render,
    pvg_render_views,
    pvg_render_semantic,
    pvg_sky_composite,
    pvg_sky_composite_views,
    l1_loss,
    pvg_ssim,
    render,
    render_bwd,
    render_features,
    render_features_bwd,
    render_fwd,
    render_views,
)
