"""FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  It shares no code with the GPU library.
"""
from .render import *  # noqa: F401,F403
from .render import Field, render_image, render_rays, bone_transforms, camera_rays  # noqa: F401
from .rng import splitmix64, stratified_xi  # noqa: F401
from .residual import hann_window, posenc, residual_offset  # noqa: F401
from .pose import refine, refined_bone_transforms  # noqa: F401
from .skel_cnn import skel_cnn_logits  # noqa: F401
from .freq_field import freq_field, posenc10  # noqa: F401
