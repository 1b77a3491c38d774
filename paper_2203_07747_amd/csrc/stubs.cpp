// (no unimplemented entry points remain)
