"""MI355X three-grid IOFD Helmholtz solver: HIP kernels behind a C ABI
(include/helm.h) with a thin ctypes binding (``paper_2608_22946_amd.helm``)."""
