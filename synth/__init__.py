"""Seeded synthetic multimodal image pairs (stand-ins for the paper's SAR/IR-optical data).

This package holds no arithmetic of the matching method itself: it only draws
scenes, warps them by a known similarity transform and applies a nonlinear
intensity remap plus multiplicative speckle.  Both the CPU oracle tests and
the GPU path take their inputs from here.
"""
from .gen import CONFIGS, make_pair, make_shifted_pair, make_scene, serving_sizes, keypoint_cap  # noqa: F401
