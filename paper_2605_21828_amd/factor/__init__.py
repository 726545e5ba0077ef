"""FP64 construction of the butterfly factor set (the input of the GPU apply): trees on the
host; column IDs on the host (build.py) or on the GPU (device_build.py, imported on use)."""
from .trees import box_bisection_tree, frequency_tree, depth_for, node_range
from .interp import column_id
from .build import build_factors
from .fourier import real_modes, FourierBlocks
