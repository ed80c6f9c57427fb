"""Small helpers shared by the tests (input shaping only)."""
import numpy as np


def leaves_from_dense(field: np.ndarray, keep=None):
    """Cut a dense (z, y, x) field (extents multiples of 8) into 8^3 leaves.
    keep: optional boolean (bz, by, bx) mask of the leaves to store.
    Returns origins (n, 3) int32 (x, y, z) and values (n, 8, 8, 8)."""
    nz, ny, nx = field.shape
    bz, by, bx = nz // 8, ny // 8, nx // 8
    leaves = field.reshape(bz, 8, by, 8, bx, 8).transpose(0, 2, 4, 1, 3, 5)
    if keep is None:
        keep = np.ones((bz, by, bx), bool)
    kz, ky, kx = np.nonzero(keep)
    origins = np.stack([kx * 8, ky * 8, kz * 8], axis=1).astype(np.int32)
    return origins, np.ascontiguousarray(leaves[kz, ky, kx])


def dense_masked(field: np.ndarray, keep: np.ndarray) -> np.ndarray:
    """The field with the voxels of dropped leaves set to zero."""
    m = np.repeat(np.repeat(np.repeat(keep, 8, 0), 8, 1), 8, 2)
    return np.where(m, field, 0).astype(field.dtype)


def rel_bound_ok(got: np.ndarray, ref: np.ndarray, scale: np.ndarray, rel: float) -> np.ndarray:
    """|got - ref| <= rel * scale, elementwise (NaN where both NaN counts as ok)."""
    both_nan = np.isnan(got) & np.isnan(ref)
    return both_nan | (np.abs(got - ref) <= rel * scale)
