"""MI355X (gfx950) state-vector library: gate sweeps, fused blocks and the
emulator shortcuts of Haener et al. (QFT as FFT, arithmetic as permutation,
measurement read off the state), behind the C ABI of include/qs.h.

``paper_1604_06460_amd.qs`` is the ctypes binding; it raises on import if the
HIP library has not been built.
"""
