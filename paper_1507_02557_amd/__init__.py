"""MI355X-native DG solver for the acoustic wave equation on hybrid meshes.

Importing the package loads nothing; ``paper_1507_02557_amd.hdg`` binds the
C-ABI library ``libhdg.so`` and ``paper_1507_02557_amd.inputs`` builds the
seeded synthetic meshes and initial data.
"""
