"""MI355X-native SKIS hot path: IIS sampling, CSR sketch, coverage estimates and greedy
max-cover behind the C-ABI library ``libskis.so`` (HIP kernels for gfx950)."""
