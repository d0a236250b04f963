"""MI355X-native BE-Index bitruss decomposition.

The compute path lives in the HIP library built from `csrc/`; `binding`
marshals arguments into its C ABI.  `synth` holds the seeded input
generators.
"""
