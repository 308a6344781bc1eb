"""MI355X-native exact kNN and friends-of-friends over a Morton plane-tree.

The HIP library (``libjz.so``) is loaded on first use by :mod:`.api`; this
package import itself loads nothing, so the input generators in
:mod:`.inputs` can be used without a GPU.
"""
__all__ = ["api", "inputs"]
