"""Linked-cell short-range forces for rigid multi-centre molecules on AMD MI355X (gfx950).

The compute path is a C-ABI shared library of hand-written HIP kernels (``libmdcell.so``);
``paper_1408_4599_amd.md`` is a thin ctypes binding to it and ``workloads`` generates seeded
synthetic scenarios.
"""
