"""Residency-octree volume ray casting on MI355X (gfx950).

The hot path lives in libresoct.so (HIP kernels behind the C ABI declared in
include/resoct.h); `resoct` is its ctypes binding and `pipeline` the host-side
frame loop (scene set-up, brick staging, plain request-driven streaming).
"""
