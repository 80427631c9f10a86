"""MI355X-native clause-trigger test (GpuShareSat's GPU clause test).

The HIP library is loaded on first use of ``paper_2012_03119_amd.gss``; importing
this package alone loads nothing, so the workload generator (``gen``) can be used
on machines without the built library.
"""
