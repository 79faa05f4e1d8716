"""HNTL search for AMD Instinct MI355X: a C-ABI HIP library (``libhntl.so``)
and its Python binding (``paper_2606_08813_amd.hntl``)."""
