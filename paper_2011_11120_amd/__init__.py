"""MI355X-native multi-dimensional convolution (MDC) and LSQR redatuming path.

`paper_2011_11120_amd.mdc` binds the HIP C-ABI library (libmdcgpu.so);
`paper_2011_11120_amd.synth` generates the seeded synthetic inputs.
"""
