"""MI355X-native leaf-patch AMR hot path (forest-of-quadtrees + wave
propagation, arXiv 1308.1472).  Import `paper_1308_1472_amd.fcx` for the
HIP library binding and `paper_1308_1472_amd.inputs` for seeded synthetic
inputs."""
