"""SparseOIT hot path on MI355X: a sort-free order-independent-transparency splat
renderer (forward and backward), active-set selection and sparse Adam, as hand-written
HIP kernels for gfx950 behind a small C ABI.

Submodules are imported on demand so that ``scenes`` (seeded inputs) loads without
the GPU library.
"""
