"""Race-free indirect-increment mesh loops on AMD MI355X (gfx950).

The compute path is libumesh.so (host planner + HIP kernels behind the C ABI
of include/umesh.h).  This package holds the ctypes binding (`umesh`), a
driver for the 2D edge-flux loop (`edgeloop`), bandwidth accounting
(`measure`) and the build script (`build`).  Importing a submodule that needs
the library raises if the library has not been built; there is no fallback.
"""
