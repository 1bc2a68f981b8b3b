"""Object-centric census stereo ranging on MI355X (gfx950).

ocsr     -- Python binding of the HIP library (libocsr.so) through its C ABI
synth    -- seeded synthetic stereo scenes and matching presets
build    -- in-tree build of libocsr.so
"""
