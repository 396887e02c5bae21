"""MI355X-native batched differentiable mesh rasterizer (HIP, gfx950).

The hot path of the differentiable mesh renderer of "Accelerating 3D Deep
Learning with PyTorch3D" (Section 3.2): coarse tile binning of a packed
heterogeneous mesh batch, a per-pixel K-nearest-faces pass producing
Fragments (face id, barycentrics, z, signed xy distance), the backward to
vertex positions, and the silhouette blend of Algorithm 1; and the point-cloud
rasterizer with Alpha and Norm compositing (Section 3.3).

The compute lives in ``librast.so`` (C ABI in include/rast.h); the Python
modules only marshal arguments:
    _lib       ctypes binding, same names as the C entry points
    raster     autograd Functions: rasterize_meshes, silhouette_blend
    points     autograd Functions: rasterize_points, alpha / norm / splat
               compositing of point clouds (Section 3.3)
    autotune   bin size / capacity / scheduler selection
    graph      hipGraph capture of forward+backward
    meshgen    seeded synthetic inputs (icospheres, packed batches)
Importing the package does not load the library; the first call does, and
raises if it is missing.
"""
__all__ = ["raster", "points", "autotune", "graph", "meshgen"]


def __getattr__(name):
    if name in ("rasterize_meshes", "silhouette_blend", "RasterSettings", "Fragments"):
        from . import raster
        return getattr(raster, name)
    raise AttributeError(name)
