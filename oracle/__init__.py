"""FP64 CPU oracle for the CCPR-FDTD path (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the product library.
"""
