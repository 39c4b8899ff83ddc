"""MI355X (gfx950) implementation of the coupled low-Mach LB-FD-PF step.

lbfd       -- ctypes binding of the C ABI (include/lbfd.h, liblbfd_hip.so)
workloads  -- seeded synthetic inputs (beds, mechanisms, configurations)
build      -- hipcc build of the library
"""
