"""MI355X-native AIREBO: HIP kernels behind a C ABI, with a thin Python binding.

Importing the package loads nothing; ``paper_1810_07026_amd.airebo`` holds the
binding and ``paper_1810_07026_amd.synth`` the seeded synthetic inputs.
"""
