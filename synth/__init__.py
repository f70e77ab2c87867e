"""Seeded synthetic depth streams shaped like hand-held RGB-D capture.

This package is the only code shared by the oracle side and the GPU side, and it
holds none of the fusion method's arithmetic: scenes are analytic solids (planes,
axis-aligned boxes, spheres), a depth frame is the camera-z of the first ray hit
per pixel, then sensor noise, dropouts and range truncation are applied. The
recordings the paper runs on (a Kinect "Teddy" sequence, section "Compilation,
UI, Usage and Examples") are not available; these streams stand in for them.
"""
from .scenes import (Scene, Stream, make_stream, render_depth, render_plane_maps, pose_look_at, colour_frames,  # noqa: F401
                     WORKLOADS, workload_params)
